"""Post-processing kernels (Gaussian convolution, effective collision
strengths, level-group sums) vs the FP64 oracle, through the C ABI.

Tolerance: the outputs are FP64 sums of at most a few thousand products of
Omega with weights that both sides form in FP64, so they agree to a few
hundred units in the last place of max|Omega|; the tests ask for 1e-12
relative to the largest value of the reference row (convolution) or pair
(Upsilon).  The group sums add the same columns in the same order as the
oracle and are compared bit for bit.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import log
from paper_1403_5524_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def nat():
    from paper_1403_5524_amd import native
    native.lib()
    return native


def _mesh(rng, m, lo, hi, uniform=False):
    if uniform:
        return np.linspace(lo, hi, m)
    E = np.sort(rng.uniform(lo, hi, m))
    E[0], E[-1] = lo, hi
    return np.unique(E)


def _omega(rng, E, P, n_res=12):
    """Smooth background plus narrow Lorentzian resonances per column."""
    bg = rng.uniform(0.1, 2.0, P)[None, :] * (1.0 + 0.3 * np.sin(E[:, None]))
    out = bg.copy()
    for _ in range(n_res):
        E0 = rng.uniform(E[0], E[-1])
        gam = rng.uniform(1e-3, 2e-2) * (E[-1] - E[0])
        amp = rng.uniform(0.5, 5.0, P)[None, :]
        out += amp * gam ** 2 / ((E[:, None] - E0) ** 2 + gam ** 2)
    return out


def _rowwise_err(got, ref):
    num = np.abs(got - ref).max(axis=-1)
    den = np.maximum(np.abs(ref).max(axis=-1), 1e-300)
    return float((num / den).max())


def _to_dev(torch, dev, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                           device=dev)


@pytest.mark.parametrize("m,P,fwhm,uniform", [
    (1000, 300, 0.012, False),   # 16 output tiles (ragged), 2 column tiles
    (777, 21, 0.05, True),       # wide band, one narrow column tile
    (130, 257, 3.0, False),      # window spans the whole mesh
    (300, 5, 1e-7, False),       # narrower than the spacing: identity
    (2, 3, 0.1, False),
])
def test_convolution_matches_oracle(torch_dev, nat, m, P, fwhm, uniform):
    torch, dev = torch_dev
    rng = np.random.default_rng(m + P)
    E = _mesh(rng, m, 0.2, 1.4, uniform)
    om = _omega(rng, E, P)
    log("convolution m=%d P=%d fwhm=%g" % (E.size, P, fwhm))
    got = nat.rm_convolve_gaussian(_to_dev(torch, dev, E),
                                   _to_dev(torch, dev, om), fwhm)
    torch.cuda.synchronize()
    ref = oracle.gaussian_convolve(E, om, fwhm)
    err = _rowwise_err(got.cpu().numpy(), ref)
    log("  max row-relative error %.2e" % err)
    assert err < TOL


def test_convolution_of_one_point(torch_dev, nat):
    torch, dev = torch_dev
    om = np.array([[0.25, -1.5, 3.0]])
    got = nat.rm_convolve_gaussian(_to_dev(torch, dev, [0.7]),
                                   _to_dev(torch, dev, om), 0.1)
    assert np.array_equal(got.cpu().numpy(), om)


def test_convolution_of_sweep_output(torch_dev, nat):
    """The sweep's own Omega(E) on the small configuration, then smoothed."""
    torch, dev = torch_dev
    w = wl.config1()
    sym = nat.load_symmetry(w.syms[0])
    E = _to_dev(torch, dev, w.mesh)
    om, _ = nat.rm_sweep_energies([sym], w.n_target, E)
    fwhm = 20.0 * (w.mesh[1] - w.mesh[0])
    sm = nat.rm_convolve_gaussian(E, om, fwhm)
    torch.cuda.synchronize()
    om_h = om.cpu().numpy()
    ref = oracle.gaussian_convolve(w.mesh, om_h, fwhm)
    err = _rowwise_err(sm.cpu().numpy().T, ref.T)   # per transition
    log("sweep output m=%d P=%d: error %.2e" % (w.mesh.size, om_h.shape[1], err))
    assert err < TOL


def test_convolution_full_size_sampled(torch_dev, nat):
    """1e5-point mesh over [0, 20] Ry, 210 transitions, FWHM 100 meV: 64
    sampled outputs, each checked against the oracle on a slice of the mesh
    that holds its whole window (a slice changes no weight inside it)."""
    torch, dev = torch_dev
    rng = np.random.default_rng(11)
    M, P = 100000, 210
    E = np.linspace(0.0, 20.0, M)
    om = _omega(rng, E, P, n_res=200)
    fwhm = 0.1 / 13.605693122994
    got = nat.rm_convolve_gaussian(_to_dev(torch, dev, E),
                                   _to_dev(torch, dev, om), fwhm)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    s = fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    idx = np.unique(np.concatenate([[0, 1, M - 2, M - 1],
                                    rng.integers(0, M, 60)]))
    worst = 0.0
    for i in idx:
        a = max(0, np.searchsorted(E, E[i] - 8 * s, side="left") - 2)
        b = min(M, np.searchsorted(E, E[i] + 8 * s, side="right") + 2)
        ref = oracle.gaussian_convolve(E[a:b], om[a:b], fwhm)[i - a]
        worst = max(worst, _rowwise_err(got[i][None], ref[None]))
    log("full-size convolution, %d sampled rows: error %.2e" % (idx.size, worst))
    assert worst < TOL


def _levels_inside(rng, n_t, lo, hi):
    """Level energies below, inside and above the mesh [lo, hi]."""
    lev = np.sort(rng.uniform(-0.2, 0.7 * hi, n_t))
    lev[0] = 0.0
    lev[-1] = hi + 0.5          # every pair with this level is closed
    if n_t > 2:
        lev[-2] = hi            # upper level exactly at the mesh top
    return lev


@pytest.mark.parametrize("m,n_t,nT,uniform", [
    (1000, 6, 11, False),     # 8 segments, two passes over temperatures
    (1501, 14, 3, True),      # 105 pairs: two column blocks
    (37, 3, 1, False),        # one segment
    (1, 2, 2, False),
])
def test_upsilon_matches_oracle(torch_dev, nat, m, n_t, nT, uniform):
    torch, dev = torch_dev
    rng = np.random.default_rng(7 * m + n_t)
    E = _mesh(rng, m, 0.05, 3.0, uniform) if m > 1 else np.array([1.0])
    P = n_t * (n_t + 1) // 2
    om = _omega(rng, E, P) if m > 1 else rng.uniform(0.5, 1.0, (1, P))
    lev = _levels_inside(rng, n_t, E[0], E[-1])
    kT = np.geomspace(0.01, 4.0, nT)
    log("upsilon m=%d n_target=%d nT=%d" % (E.size, n_t, nT))
    got = nat.rm_effective_collision_strengths(
        _to_dev(torch, dev, E), _to_dev(torch, dev, om), lev, n_t, kT)
    ref = oracle.effective_collision_strengths(E, om, lev, n_t, kT)
    got = got.cpu().numpy()
    closed = ref.max(axis=1) == 0.0
    assert np.all(got[closed] == 0.0)
    err = _rowwise_err(got[~closed], ref[~closed]) if (~closed).any() else 0.0
    log("  max pair-relative error %.2e" % err)
    assert err < TOL


def test_upsilon_full_size(torch_dev, nat):
    """1e5-point mesh, 20 levels (210 pairs), 8 temperatures: every pair."""
    torch, dev = torch_dev
    rng = np.random.default_rng(5)
    M, n_t = 100000, 20
    E = np.linspace(0.0, 20.0, M)
    P = n_t * (n_t + 1) // 2
    om = _omega(rng, E, P, n_res=200)
    lev = np.sort(rng.uniform(0.0, 12.0, n_t))
    lev[0] = 0.0
    kT = np.geomspace(0.02, 10.0, 8)
    got = nat.rm_effective_collision_strengths(
        _to_dev(torch, dev, E), _to_dev(torch, dev, om), lev, n_t, kT)
    ref = oracle.effective_collision_strengths(E, om, lev, n_t, kT)
    err = _rowwise_err(got.cpu().numpy(), ref)
    log("full-size upsilon: error %.2e" % err)
    assert err < TOL


@pytest.mark.parametrize("m,n_t,n_g", [
    (513, 14, 5), (3, 1, 1), (70, 9, 9),
    (40, 100, 7),     # 5050 transitions: rows staged in column chunks
    (9, 95, 92),      # more group pairs than the LDS accumulator holds
])
def test_group_sums_bit_exact(torch_dev, nat, m, n_t, n_g):
    torch, dev = torch_dev
    rng = np.random.default_rng(m + 31 * n_t)
    P = n_t * (n_t + 1) // 2
    om = rng.normal(size=(m, P))
    group = rng.integers(0, n_g, n_t)
    if n_g == n_t:
        group = rng.permutation(n_t)
    log("group sums m=%d n_target=%d n_group=%d" % (m, n_t, n_g))
    got = nat.rm_group_collision_strengths(_to_dev(torch, dev, om), n_t,
                                           group, n_g)
    ref = oracle.group_collision_strengths(om, n_t, group, n_g)
    assert np.array_equal(got.cpu().numpy(), ref)
