"""Pins of the oracle's channel functions (open: Coulomb F, G; closed:
decaying Whittaker) against library routines, closed forms and identities."""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import coulomb as oc


def _mp_fg(l, eta, rho):
    """F, F', G, G' at 30 digits; derivatives from A&S 14.2.2."""
    with mpmath.workdps(30):
        e, r = mpmath.mpf(eta), mpmath.mpf(rho)
        F0, G0 = mpmath.coulombf(l, e, r), mpmath.coulombg(l, e, r)
        F1, G1 = mpmath.coulombf(l + 1, e, r), mpmath.coulombg(l + 1, e, r)
        S = (l + 1) / r + e / (l + 1)
        R = mpmath.sqrt((l + 1) ** 2 + e * e) / (l + 1)
        return [float(v) for v in (F0, S * F0 - R * F1, G0, S * G0 - R * G1)]


def test_steed_matches_mpmath():
    """Steed's CF1/CF2 branch against mpmath.coulombf/coulombg (DLMF 33.2),
    beyond the turning point (the domain met at r = a)."""
    rng = np.random.default_rng(5)
    cases = []
    while len(cases) < 24:
        l = int(rng.integers(0, 6))
        eta = float(rng.choice([-60.0, -8.0, -1.3, -0.2, 0.0, 0.7, 2.5]))
        rho = float(np.exp(rng.uniform(np.log(0.4), np.log(90.0))))
        if rho > 1.05 * (eta + math.sqrt(eta * eta + l * (l + 1))):
            cases.append((l, eta, rho))
    for l, eta, rho in cases:
        ref = _mp_fg(l, eta, rho)
        got = oracle.coulomb_fg(l, eta, rho)
        scale = max(abs(ref[0]), abs(ref[2]))
        dscale = max(abs(ref[1]), abs(ref[3]))
        for r_, g_, sc in zip(ref, got, (scale, dscale, scale, dscale)):
            assert abs(float(g_) - r_) <= 1e-12 * sc, (l, eta, rho, r_, g_)


def test_neutral_reduces_to_riccati_bessel():
    """z = 0: F_l = rho j_l(rho), G_l = -rho y_l(rho) (A&S 14.6.4)."""
    for l in range(6):
        rho = np.linspace(1.05 * math.sqrt(l * (l + 1)) + 0.3, 60.0, 37)
        F, Fp, G, Gp = oracle.coulomb_fg(np.full(rho.size, l), 0.0, rho)
        jl, yl = sp.spherical_jn(l, rho), sp.spherical_yn(l, rho)
        jp = sp.spherical_jn(l, rho, derivative=True)
        yp = sp.spherical_yn(l, rho, derivative=True)
        np.testing.assert_allclose(F, rho * jl, rtol=0, atol=1e-13 * np.abs(
            rho * yl).max())
        np.testing.assert_allclose(G, -rho * yl, rtol=1e-12)
        np.testing.assert_allclose(Fp, jl + rho * jp, rtol=0, atol=1e-12)
        np.testing.assert_allclose(Gp, -(yl + rho * yp), rtol=1e-11)


def test_wronskian_all_branches():
    """F'G - FG' = 1 (DLMF 33.2.13), Steed and near-threshold branches."""
    k = np.array([3.0, 1.0, 0.3, 0.05, 0.011, 0.009, 2e-3, 1e-4])
    for l in (0, 3, 5):
        s, c, spr, cpr = oracle.open_channel_functions(np.full(k.size, l),
                                                       1.0, k, 20.0)
        np.testing.assert_allclose(c * spr - s * cpr, 1.0, rtol=0, atol=1e-11)


def test_open_functions_continuous_across_branch_switch():
    """The |eta| = 100 switch between Steed and mpmath is seamless."""
    kc = 1.0 / oc.ETA_STEED
    k = np.array([kc * (1 - 1e-7), kc * (1 + 1e-7)])
    for l in (0, 2, 5):
        vals = oracle.open_channel_functions(np.full(2, l), 1.0, k, 20.0)
        for v in vals:
            assert abs(v[0] - v[1]) <= 1e-6 * max(1.0, abs(v[0]))


def test_open_functions_finite_threshold_limit():
    """k^-1/2 F and k^-1/2 G tend to finite limits as E -> threshold+
    (attractive Coulomb); successive decades differ by O(k^2)."""
    k = np.array([1e-2, 1e-3, 1e-4])
    s, c, spr, cpr = oracle.open_channel_functions(np.full(3, 5), 1.0, k, 20.0)
    assert np.all(np.isfinite(s)) and np.all(np.isfinite(c))
    assert abs(s[2] - s[1]) < 1e-4 * abs(s[1])
    assert abs(c[2] - c[1]) < 1e-4 * abs(c[1])
    assert abs(s[1] - s[0]) > abs(s[2] - s[1])


def _mp_whit_L(kappa, l, x):
    with mpmath.workdps(30):
        W = lambda y: mpmath.whitw(kappa, l + 0.5, y)
        return float(x * mpmath.diff(W, x) / W(x))


def test_closed_cf_matches_mpmath_whitw():
    """Continued-fraction branch against mpmath.whitw (DLMF 13.14)."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        phi = float(np.exp(rng.uniform(np.log(1.0 / oc.KAPPA_CF), np.log(1.5))))
        l = int(rng.integers(0, 6))
        L = oracle.closed_channel_logderiv(l, 1.0, phi, 20.0)
        ref = _mp_whit_L(1.0 / phi, l, 40.0 * phi)
        assert abs(math.atan(float(L)) - math.atan(ref)) < 1e-12, (phi, l)


def test_closed_neutral_reduces_to_bessel_k():
    """z = 0: W_{0,mu}(x) = sqrt(x/pi) K_mu(x/2) (DLMF 13.18.9)."""
    phi = np.array([0.05, 0.3, 1.0, 1.4])
    for l in range(6):
        L = oracle.closed_channel_logderiv(np.full(4, l), 0.0, phi, 20.0)
        x = 2 * phi * 20.0
        ref = 0.5 + 0.5 * x * sp.kvp(l + 0.5, x / 2) / sp.kv(l + 0.5, x / 2)
        np.testing.assert_allclose(L, ref, rtol=1e-12)


@pytest.mark.parametrize("n,l", [(3, 0), (5, 2), (7, 5), (12, 1), (40, 3)])
def test_closed_hydrogenic_closed_form(n, l):
    """Integer kappa = n > l: W_{n,l+1/2}(x) is proportional to
    x^(l+1) exp(-x/2) L^(2l+1)_{n-l-1}(x) (DLMF 13.18.17)."""
    phi = 1.0 / n
    x = 40.0 * phi
    m = n - l - 1
    lag = sp.eval_genlaguerre(m, 2 * l + 1, x)
    dlag = -sp.eval_genlaguerre(m - 1, 2 * l + 2, x) if m > 0 else 0.0
    ref = (l + 1) - x / 2 + x * dlag / lag
    L = float(oracle.closed_channel_logderiv(l, 1.0, phi, 20.0))
    assert abs(math.atan(L) - math.atan(ref)) < 1e-11


def test_closed_continuous_across_branch_switch():
    kap = oc.KAPPA_CF
    phi = np.array([1.0 / (kap * (1 - 1e-8)), 1.0 / (kap * (1 + 1e-8))])
    for l in (0, 3, 5):
        L = oracle.closed_channel_logderiv(np.full(2, l), 1.0, phi, 20.0)
        assert abs(L[0] - L[1]) < 1e-5 * max(1.0, abs(L[0]))
