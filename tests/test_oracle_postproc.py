"""Pins of the post-processing oracle (Gaussian convolution of Omega(E) and
Maxwellian-averaged effective collision strengths) against closed forms.
CPU only."""
import numpy as np
import pytest

import oracle


def _nonuniform_mesh(rng, m, lo, hi):
    x = np.sort(rng.uniform(lo, hi, m))
    return np.unique(x)


def test_convolution_keeps_constants_on_any_mesh():
    rng = np.random.default_rng(0)
    E = _nonuniform_mesh(rng, 400, 0.0, 2.0)
    om = np.tile(np.array([1.5, -0.25, 3.0]), (E.size, 1))
    out = oracle.gaussian_convolve(E, om, fwhm=0.05)
    assert np.abs(out - om).max() < 1e-14


def test_convolution_of_gaussians_widths_add_in_quadrature():
    """A Gaussian of width s1 convolved with one of width s2 (unit area) is
    the Gaussian of width sqrt(s1^2 + s2^2) with amplitude s1/sqrt(...)."""
    E = np.linspace(0.0, 2.0, 20001)           # h = 1e-4
    s1, fwhm = 0.02, 0.03
    s2 = fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    E0 = 1.0
    om = np.exp(-0.5 * ((E - E0) / s1) ** 2)[:, None]
    out = oracle.gaussian_convolve(E, om, fwhm)[:, 0]
    st = np.hypot(s1, s2)
    ref = (s1 / st) * np.exp(-0.5 * ((E - E0) / st) ** 2)
    inner = (E > 0.5) & (E < 1.5)
    assert np.abs(out[inner] - ref[inner]).max() < 1e-8


def test_convolution_keeps_linear_functions_in_the_interior():
    E = np.linspace(0.0, 1.0, 2001)
    om = (0.3 + 2.0 * E)[:, None]
    out = oracle.gaussian_convolve(E, om, fwhm=0.02)
    s = 0.02 / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    inner = (E > 8 * s + 1e-12) & (E < 1.0 - 8 * s - 1e-12)
    assert np.abs(out[inner, 0] - om[inner, 0]).max() < 1e-12


def test_convolution_narrow_kernel_is_identity():
    """A width far below the mesh spacing leaves every point alone."""
    rng = np.random.default_rng(1)
    E = _nonuniform_mesh(rng, 300, 0.0, 1.0)
    om = rng.normal(size=(E.size, 2))
    out = oracle.gaussian_convolve(E, om, fwhm=1e-9)
    assert np.abs(out - om).max() <= 1e-15 * np.abs(om).max()


def _upsilon_const(c, X):
    return c * (1.0 - np.exp(-X))


@pytest.mark.parametrize("kT", [0.05, 0.3, 2.0])
def test_upsilon_of_constant_omega(kT):
    """Omega = c above threshold: Upsilon = c (1 - exp(-eps_max / kT))."""
    e_level = np.array([0.0, 0.4])
    E = 0.4 + 1e-9 + np.linspace(0.0, 3.0, 30001)   # eps from ~0 to 3
    om = np.zeros((E.size, 3))
    om[:, 1] = 2.5                                   # pair (0, 1)
    ups = oracle.effective_collision_strengths(E, om, e_level, 2, [kT])
    X = (E[-1] - 0.4) / kT
    # trapezoid error of exp(-x) with step h/kT: ~ X (h/kT)^2 / 12
    h = (E[1] - E[0]) / kT
    assert abs(ups[1, 0] - _upsilon_const(2.5, X)) < 2.5 * h * h + 1e-12


def test_upsilon_of_linear_omega():
    """Omega = a + b eps: Upsilon = a (1 - e^-X) + b kT (1 - (1 + X) e^-X)."""
    a, b, kT = 0.7, 1.3, 0.25
    e_level = np.array([0.1, 0.0, 0.6])
    n_t = 3
    e = 0.6                                           # pairs with level 2
    E = e + 1e-9 + np.linspace(0.0, 4.0, 40001)
    eps = E - e
    P = n_t * (n_t + 1) // 2
    om = np.zeros((E.size, P))
    p = 1 * n_t - 0 + (2 - 1)                         # pair (1, 2)
    om[:, p] = a + b * eps
    ups = oracle.effective_collision_strengths(E, om, e_level, n_t, [kT])
    X = eps[-1] / kT
    ref = a * (1 - np.exp(-X)) + b * kT * (1 - (1 + X) * np.exp(-X))
    h = (E[1] - E[0]) / kT
    assert abs(ups[p, 0] - ref) < 10 * h * h


def test_upsilon_pair_columns_and_closed_pairs():
    """Each packed column feeds its own level pair; a pair whose upper level
    lies above the mesh gets 0."""
    n_t = 3
    e_level = np.array([0.0, 0.2, 5.0])
    E = np.linspace(0.3, 2.0, 5001)
    P = n_t * (n_t + 1) // 2
    cols = np.arange(1, P + 1, dtype=np.float64)
    om = np.tile(cols, (E.size, 1))
    ups = oracle.effective_collision_strengths(E, om, e_level, n_t, [0.5])
    for t in range(n_t):
        for u in range(t, n_t):
            p = oracle.omega_pair_index(t, u, n_t)
            e = max(e_level[t], e_level[u])
            if e >= E[-1]:
                assert ups[p, 0] == 0.0
            else:
                X = (E[-1] - e) / 0.5
                x0 = (E[0] - e) / 0.5       # first mesh point above e
                # constant Omega: c (1 - e^-x0) + trapezoid of c e^-x on
                # [x0, X], which tends to c (e^-x0 - e^-X)
                assert abs(ups[p, 0] - cols[p] * (1 - np.exp(-X))) < 1e-6 * cols[p]


def test_convolution_of_one_point_mesh_is_identity():
    om = np.array([[0.5, -2.0]])
    assert np.array_equal(oracle.gaussian_convolve(np.array([1.0]), om, 0.1), om)


def _full_symmetric(om_row, n_t):
    """Packed upper triangle -> full symmetric n_t x n_t matrix."""
    F = np.zeros((n_t, n_t))
    for t in range(n_t):
        for u in range(t, n_t):
            F[t, u] = F[u, t] = om_row[oracle.omega_pair_index(t, u, n_t)]
    return F


def test_grouping_by_ordered_pair_sums():
    """Brute force over ordered level pairs: for a != b the block sum of the
    full symmetric matrix; for a == b half of the block sum plus half of its
    diagonal (each unordered pair once, elastic ones included)."""
    rng = np.random.default_rng(3)
    n_t, n_g = 7, 3
    group = np.array([2, 0, 1, 0, 2, 2, 1])
    P = n_t * (n_t + 1) // 2
    om = rng.uniform(0.0, 1.0, size=(4, P))
    out = oracle.group_collision_strengths(om, n_t, group, n_g)
    for i in range(om.shape[0]):
        F = _full_symmetric(om[i], n_t)
        for a in range(n_g):
            for b in range(a, n_g):
                ia, ib = np.where(group == a)[0], np.where(group == b)[0]
                blk = F[np.ix_(ia, ib)]
                ref = blk.sum() if a != b else 0.5 * (blk.sum() + np.trace(blk))
                q = oracle.omega_pair_index(a, b, n_g)
                assert abs(out[i, q] - ref) < 1e-14 * max(1.0, abs(ref))


def test_grouping_identity_and_total():
    rng = np.random.default_rng(4)
    n_t = 5
    P = n_t * (n_t + 1) // 2
    om = rng.normal(size=(3, P))
    same = oracle.group_collision_strengths(om, n_t, np.arange(n_t), n_t)
    assert np.array_equal(same, om)
    one = oracle.group_collision_strengths(om, n_t, np.zeros(n_t, int), 1)
    assert np.allclose(one[:, 0], om.sum(axis=1), rtol=0, atol=1e-13)
