"""Resonance pins of the oracle (single channel): the K-matrix against the
Lane-Thomas closed form, and an isolated narrow pole against Breit-Wigner.

With rho = k a and Coulomb functions from mpmath, the penetration factor
P = rho/(F^2 + G^2), shift factor S = rho (F F' + G G')/(F^2 + G^2) and
hard-sphere phase phi = atan2(F, G) give, for a one-channel R-matrix R(E)
(Bloch constant 0), tan(delta + phi) = P R / (1 - S R) with K = tan(delta)
(Lane & Thomas, Rev. Mod. Phys. 30 (1958) 257).  For one pole,
R = gamma^2/(E_l - E) with gamma^2 = w^2/(2a), the resonance sits at
E_r = E_l - S gamma^2 with width Gamma = 2 P gamma^2.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle

A = 20.0


def _pso(l, z, E):
    k = math.sqrt(E)
    with mpmath.workdps(30):
        eta, rho = -z / mpmath.mpf(k), mpmath.mpf(k) * A
        F, G = mpmath.coulombf(l, eta, rho), mpmath.coulombg(l, eta, rho)
        Fp = mpmath.diff(lambda x: mpmath.coulombf(l, eta, x), rho)
        Gp = mpmath.diff(lambda x: mpmath.coulombg(l, eta, x), rho)
        d = F * F + G * G
        return (float(rho / d), float(rho * (F * Fp + G * Gp) / d),
                float(mpmath.atan2(F, G)))


def _K(sym, E):
    return np.array([oracle.sweep(sym, [e], keep=("K",))["K"][0][0][0, 0]
                     for e in E])


@pytest.mark.parametrize("l", [0, 3])
def test_single_channel_k_matches_lane_thomas(l):
    rng = np.random.default_rng(4)
    Ek = np.sort(rng.uniform(-1.0, 30.0, 60))
    w = rng.normal(0, 0.3, (1, 60))
    sym = {"E_pole": Ek, "w": w, "a": A, "e_thr": np.array([0.0]),
           "l": np.array([l]), "z": 1.0, "g": 1.0, "target": None}
    for E in (0.37, 2.9, 7.3):
        R = oracle.r_matrix(Ek, w, A, [E])[0, 0, 0]
        P, S, phi = _pso(l, 1.0, E)
        K = _K(sym, [E])[0]
        delta = math.atan(K)
        t = math.tan(delta + phi)
        ref = P * R / (1.0 - S * R)
        assert abs(t - ref) <= 1e-9 * max(1.0, abs(ref))


def test_isolated_pole_breit_wigner_width_and_position():
    l, z, El, c = 0, 1.0, 3.0, 2e-3
    g2 = c * c / (2 * A)
    sym = {"E_pole": np.array([El]), "w": np.array([[c]]), "a": A,
           "e_thr": np.array([0.0]), "l": np.array([l]), "z": z, "g": 1.0,
           "target": None}
    P, S, _ = _pso(l, z, El)
    Gam = 2 * P * g2
    Er = El - S * g2
    E = Er + Gam * np.linspace(-20, 20, 801)
    d = np.unwrap(2 * np.arctan(_K(sym, E))) / 2
    rise = d[-1] - d[0]
    assert abs(rise - 2 * math.atan(40.0)) < 1e-2
    slope = np.gradient(d, E)
    i = int(np.argmax(slope))
    assert abs(E[i] - Er) < 0.06 * Gam
    assert abs(2.0 / slope[i] - Gam) < 1e-2 * Gam


def test_measured_resonance_matches_lane_thomas():
    """oracle.resonance.measure_resonance on the isolated pole above: the
    slope of the eigenphase sum gives the Lane-Thomas position and width
    (E_l - S gamma^2, 2 P gamma^2, mpmath Coulomb functions) to 1 %, for
    widths from 1e-5 to 1e-3 Ry, starting from the pole energy."""
    from oracle import resonance
    l, z, El = 0, 1.0, 3.0
    P, S, _ = _pso(l, z, El)
    for Gam_target in (1e-5, 1e-4, 1e-3):
        g2 = Gam_target / (2 * P)
        c = math.sqrt(2 * A * g2)
        sym = {"E_pole": np.array([El]), "w": np.array([[c]]), "a": A,
               "e_thr": np.array([0.0]), "l": np.array([l]), "z": z,
               "g": 1.0, "target": None}
        Er, Gam = resonance.measure_resonance(sym, El, 0.05)
        assert abs(Gam - 2 * P * g2) < 1e-2 * Gam
        assert abs(Er - (El - S * g2)) < 2e-2 * Gam


def test_measured_resonance_in_a_coupled_system_is_the_decoupled_one():
    """A narrow pole coupled to one channel of a 3-channel system whose
    background poles couple the channels: measured in the full system it
    agrees, within 5 % of its width, with the same pole measured in the
    one-channel system of that channel alone plus the background poles'
    diagonal (R of the other channels does not reach a pole that couples
    to nothing else at first order).  A planted mistake in the measurement
    (the slope without unwrapping, or 1/slope for the width) fails."""
    from oracle import resonance
    rng = np.random.default_rng(9)
    nh = 40
    Ek = np.sort(rng.uniform(-2.0, 30.0, nh))
    w = np.zeros((3, nh))
    w[:, :] = rng.normal(0.0, 0.02, (3, nh))
    El = 6.1234
    E_all = np.sort(np.concatenate([Ek, [El]]))
    k = int(np.searchsorted(E_all, El))
    w_all = np.insert(w, k, 0.0, axis=1)
    w_all[0, k] = 0.02
    sym = {"E_pole": E_all, "w": w_all, "a": A,
           "e_thr": np.array([0.0, 0.5, 1.0]), "l": np.array([0, 1, 2]),
           "z": 1.0, "g": 1.0, "target": None}
    Er, Gam = resonance.measure_resonance(sym, El, 0.05)
    one = {"E_pole": E_all, "w": w_all[:1], "a": A, "e_thr": np.array([0.0]),
           "l": np.array([0]), "z": 1.0, "g": 1.0, "target": None}
    Er1, Gam1 = resonance.measure_resonance(one, El, 0.05)
    assert 1e-5 < Gam < 1e-2
    assert abs(Gam - Gam1) < 0.05 * Gam1
    assert abs(Er - Er1) < 0.05 * Gam1
    # planted: width from the slope itself instead of 2 / slope
    E = np.linspace(Er - 4 * Gam, Er + 4 * Gam, 41)
    d = resonance.eigenphase_sum(sym, E)
    s = np.max(np.diff(np.unwrap(2 * d) / 2) / (E[1] - E[0]))
    assert abs(1.0 / s - Gam) > 0.3 * Gam
