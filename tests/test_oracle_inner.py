"""Pins of the inner-region oracle (model Hamiltonian in the Bloch sine
basis, full eigen-solve): the square well, the low poles of an independent
polynomial basis, and R(E) from the poles against direct integration.
CPU only."""
import numpy as np
import pytest

from oracle import inner
from model_systems import ModelSystem, bloch_poles, ode_rmatrix


def _model(n, e, l, z, a, depth, rng_):
    return {"e_thr": np.asarray(e, float), "l": np.asarray(l), "z": z, "a": a,
            "depth": np.asarray(depth, float), "range": np.asarray(rng_, float)}


def _as_system(m):
    D, Rg = m["depth"], m["range"]
    return ModelSystem(m["e_thr"], m["l"], m["z"], m["a"],
                       lambda r: -D * np.exp(-(r / Rg) ** 2))


def test_square_well_poles_and_amplitudes():
    """Constant potential -V0 (a Gaussian of enormous range): the basis is
    the eigenbasis, E_m = kappa_m^2 - V0, |w_m| = 2 / sqrt(a)."""
    a, V0, N = 7.0, 1.3, 60
    m = _model(1, [0.0], [0], 0.0, a, [[V0]], [[1e9]])
    E, w = inner.inner_region(m, N, Q=3 * N)
    kap = (np.arange(N) + 0.5) * np.pi / a
    assert np.abs(E - (kap ** 2 - V0)).max() < 1e-10 * kap[-1] ** 2
    assert np.abs(np.abs(w[0]) - 2.0 / np.sqrt(a)).max() < 1e-10


def test_low_poles_agree_with_polynomial_basis():
    """Two coupled channels with Coulomb and centrifugal terms: the lowest
    poles from the sine basis and from the independent polynomial basis
    r P_m(2r/a - 1) (same Bloch problem, b = 0) agree once both converge
    (the sine basis converges as 1/N^3 here: 2.2e-5, 2.8e-6, 3.6e-7 on the
    lowest pole at N = 160, 320, 640)."""
    m = _model(2, [0.0, 0.3], [0, 1], 1.0, 8.0,
               [[2.0, 0.6], [0.6, 1.4]], [[2.5, 3.0], [3.0, 2.0]])
    E, _ = inner.inner_region(m, 640, Q=1380)
    Ep, _ = bloch_poles(_as_system(m), N=60)
    k = 8
    assert np.abs(E[:k] - np.sort(Ep)[:k]).max() < 1e-6 * max(1.0, np.abs(E[:k]).max())


@pytest.mark.parametrize("E", [0.45, 1.7])
def test_rmatrix_from_poles_against_direct_integration(E):
    """R(E) = (1/2a) sum_k w w / (E_k - E) from the computed poles, plus the
    free tail of the basis states left out, against the R-matrix of direct
    integration (two l = 0 channels, Gaussian couplings, no Coulomb)."""
    a, N = 6.0, 240
    m = _model(2, [0.0, 0.25], [0, 0], 0.0, a,
               [[1.5, 0.5], [0.5, 0.9]], [[2.0, 2.5], [2.5, 1.8]])
    Ek, w = inner.inner_region(m, N, Q=N + 200)
    R = (w / (Ek - E)) @ w.T / (2.0 * a)
    kap = (np.arange(N, N + 2000000) + 0.5) * np.pi / a
    for i, e in enumerate(m["e_thr"]):
        R[i, i] += (2.0 / a ** 2) * np.sum(1.0 / (kap ** 2 + e - E))
    Rref = ode_rmatrix(_as_system(m), E)
    assert np.abs(R - Rref).max() < 2e-5 * np.abs(Rref).max()


@pytest.mark.parametrize("Q", [1, 2, 7, 50])
def test_quadrature_is_gauss_legendre(Q):
    """Nodes and weights on [0, a] agree with numpy's Gauss-Legendre rule
    mapped there (absolute, in x), and integrate r^k exactly for k < 2Q."""
    from numpy.polynomial import legendre as npleg
    a = 3.0
    r, w = inner.quadrature(a, Q)
    x, wl = npleg.leggauss(Q)
    assert np.abs((2.0 * r / a - 1.0) - x).max() < 4e-16
    assert np.abs(2.0 * w / a - wl).max() < 1e-14
    for k in range(2 * Q):
        exact = a ** (k + 1) / (k + 1)
        assert abs(np.sum(w * r ** k) - exact) < 1e-13 * exact


@pytest.mark.parametrize("Q,nodes", [(50, range(50)), (400, (0, 1, 2, 200)),
                                     (1000, (0, 1)), (4000, (0,))])
def test_quadrature_nodes_relative_accuracy(Q, nodes):
    """Next to r = 0 each node must carry full relative accuracy (the
    centrifugal term scales as 1/r^2 there): the zeros of P_Q and their
    weights 2 / ((1 - x^2) P_Q'(x)^2) from mpmath at 40 digits, compared as
    r = 1 + x on [0, 2].  (Forming 1 - cos(theta) instead of 2 sin^2(theta/2)
    is off by 1.5e-13 at Q = 4000.)"""
    import mpmath as mp
    r, w = inner.quadrature(2.0, Q)
    with mp.workdps(40):
        f = lambda x: mp.re(mp.legendre(Q, x))
        for k in nodes:
            xk = mp.re(mp.findroot(f, mp.mpf(float(r[k])) - 1,
                                   tol=mp.mpf(10) ** -60))
            dp = mp.re(mp.diff(f, xk))
            rk = 1 + xk
            wk = 2 / ((1 - xk * xk) * dp * dp)
            assert abs(float((r[k] - rk) / rk)) < 1e-14
            assert abs(float((w[k] - wk) / wk)) < 1e-14


def test_pure_coulomb_gives_the_hydrogen_levels():
    """z = 1 and no short-range potential: the lowest poles in a box of
    a = 40 a0 are the hydrogenic levels -z^2/n^2 Ry (1s, 2s; 2p, 3p), the
    box and the 1/r cusp moving them by less than 2e-5 at N = 800 (l = 0)
    and 400 (l = 1); the 1s error falls as N^-3 (ratio ~8 per doubling)."""
    def levels(l, N):
        m = _model(1, [0.0], [l], 1.0, 40.0, [[0.0]], [[1.0]])
        return inner.inner_region(m, N, Q=2 * N + 100)[0]
    E400, E800 = levels(0, 400), levels(0, 800)
    assert np.abs(E800[:2] - np.array([-1.0, -0.25])).max() < 2e-5
    r = (E400[0] + 1.0) / (E800[0] + 1.0)
    assert 6.0 < r < 10.0
    Ep = levels(1, 400)
    assert np.abs(Ep[:2] - np.array([-0.25, -1.0 / 9.0])).max() < 5e-6
