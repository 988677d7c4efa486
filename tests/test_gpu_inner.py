"""Inner-region eigen-solve through the C ABI vs the FP64 oracle (needs an
MI355X).

Both sides assemble H by a Q-point quadrature (elements differing by the
rounding of Q-term sums) and diagonalise it with a backward-stable
eigen-solver (the exact eigenpairs of H + dH, |dH| of order D eps S; D the
dimension, S the spectrum's scale).  Every tolerance follows from one budget
eta = 8 (D + Q) eps S for the difference of the two:
* eigenvalues (unique): |dE_k| <= eta (Weyl);
* amplitudes: the sign of an eigenvector and the basis of a degenerate
  eigenspace are not unique, so w is compared up to sign, for poles whose
  gap g_k to their neighbours exceeds 1e-6 S, within f sqrt(N) eta / g_k
  (Davis-Kahan; f = 2/sqrt(a) maps an eigenvector to its amplitude);
* R(E) = (1/2a) sum_k w w / (E_k - E) (invariant): first-order perturbation
  of (1/2a) B (H - E)^-1 B^T gives |dR_ij| <= (eta/2a) sqrt(G_i G_j),
  G_i = sum_k w_ik^2 / (E_k - E)^2, at energies between the poles;
* Omega from a full sweep over the poles: normwise 1e-6, the path's FP64
  bound."""
import time

import numpy as np
import pytest

import oracle
from oracle import inner
from gpu_helpers import log, omega_normwise_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nat():
    import torch
    assert torch.cuda.is_available()
    from paper_1403_5524_amd import native
    native.lib()
    return native


def _model(e, l, z, a, depth, rng_):
    return {"e_thr": np.asarray(e, float), "l": np.asarray(l), "z": z, "a": a,
            "depth": np.asarray(depth, float), "range": np.asarray(rng_, float)}


def _random_model(n, seed, a=8.0, z=1.0):
    rng = np.random.default_rng(seed)
    D = rng.uniform(0.2, 1.0, (n, n))
    D = 0.5 * (D + D.T) + np.diag(rng.uniform(0.8, 2.5, n))
    Rg = rng.uniform(1.5, 3.5, (n, n))
    Rg = 0.5 * (Rg + Rg.T)
    e = np.sort(rng.uniform(0.0, 0.8, n))
    e[0] = 0.0
    return _model(e, rng.integers(0, 3, n), z, a, D, Rg)


def _compare(nat, m, N, Q=None, check_w=True):
    """Largest ratio of each difference to its bound: (E, w, R, sweeps)."""
    t0 = time.perf_counter()
    Eg, wg, sweeps, _ = nat.rm_inner_region(m, N, Q or 0)
    log("  device solve D=%d: %.3f s" % (Eg.size, time.perf_counter() - t0))
    Eo, wo = inner.inner_region(m, N, Q)
    assert np.all(np.diff(Eg) >= 0.0)
    D = Eo.size
    S = max(np.abs(Eo).max(), 1.0)
    Qn = Q or N + 48
    eta = 8.0 * (D + Qn) * np.finfo(float).eps * S
    e_ratio = np.abs(Eg - Eo).max() / eta
    a = m["a"]
    w_ratio = 0.0
    if check_w and D > 1:
        gap = np.full(D, np.inf)
        d = np.diff(Eo)
        gap[:-1] = d
        gap[1:] = np.minimum(gap[1:], d)
        sel = gap > 1e-6 * S
        diff = np.minimum(np.abs(wg - wo), np.abs(wg + wo)).max(axis=0)
        bound = 2.0 / np.sqrt(a) * np.sqrt(N) * eta / gap
        if sel.any():
            w_ratio = (diff[sel] / bound[sel]).max()
    k = min(D, 12)
    Es = [Eo[0] - 0.5] + [0.5 * (Eo[i] + Eo[i + 1]) for i in range(k - 1)
                          if Eo[i + 1] - Eo[i] > 1e-6 * S]
    r_ratio = 0.0
    for E in Es:
        Rg = (wg / (Eg - E)) @ wg.T / (2.0 * a)
        Ro = oracle.r_matrix(Eo, wo, a, E)[0]
        G = np.sqrt(((wo / (Eo - E)) ** 2).sum(axis=1))
        bound = eta / (2.0 * a) * np.outer(G, G)
        r_ratio = max(r_ratio, (np.abs(Rg - Ro) / bound).max())
    return e_ratio, w_ratio, r_ratio, sweeps


def _log_and_check(name, errs):
    e_r, w_r, r_r, sweeps = errs
    log("%s: sweeps %d, error / bound: E %.2e, w %.2e, R %.2e"
        % (name, sweeps, e_r, w_r, r_r))
    assert e_r < 1.0 and w_r < 1.0 and r_r < 1.0


def test_square_well_is_the_basis(nat):
    """Constant potential: E_m = kappa_m^2 - V0 and |w_m| = 2/sqrt(a)."""
    a, V0, N = 7.0, 1.3, 60
    m = _model([0.0], [0], 0.0, a, [[V0]], [[1e9]])
    E, w, _, _ = nat.rm_inner_region(m, N, 3 * N)
    kap = (np.arange(N) + 0.5) * np.pi / a
    assert np.abs(E - (kap ** 2 - V0)).max() < 1e-11 * kap[-1] ** 2
    assert np.abs(np.abs(w[0]) - 2.0 / np.sqrt(a)).max() < 1e-10


def test_two_coupled_channels(nat):
    m = _model([0.0, 0.3], [0, 1], 1.0, 8.0,
               [[2.0, 0.6], [0.6, 1.4]], [[2.5, 3.0], [3.0, 2.0]])
    _log_and_check("n=2 N=40", _compare(nat, m, 40))


@pytest.mark.parametrize("n,N", [(1, 1), (1, 2), (2, 1), (3, 15), (5, 13)])
def test_small_and_odd_dimensions(nat, n, N):
    """D = n N of 1, 2, 45 and 65: a single column, the padding column of an
    odd dimension, ragged pair counts."""
    _log_and_check("n=%d N=%d" % (n, N), _compare(nat, _random_model(n, 10 + n * N), N))


def test_degenerate_channels(nat):
    """Two identical uncoupled channels: every pole doubly degenerate, so
    only the invariants are compared."""
    m = _model([0.2, 0.2], [1, 1], 1.0, 6.0, [[1.1, 0.0], [0.0, 1.1]],
               [[2.0, 1.0], [1.0, 2.0]])
    _log_and_check("degenerate", _compare(nat, m, 30, check_w=False))


def test_several_blocks(nat):
    """D = 1024: 512 column pairs per step, 128 workgroups."""
    _log_and_check("n=4 N=256", _compare(nat, _random_model(4, 3), 256))


def test_maximum_dimension(nat):
    """D = 4096, the largest size compared with the oracle's full eigen-solve."""
    _log_and_check("n=2 N=2048", _compare(nat, _random_model(2, 4), 2048))


def test_sweep_over_the_inner_region_poles(nat):
    """Poles from the device solve loaded and swept give the Omega of the
    oracle's poles swept by the oracle."""
    import torch
    m = _random_model(3, 7, a=10.0)
    N = 120
    Eg, wg, _, _ = nat.rm_inner_region(m, N)
    Eo, wo = inner.inner_region(m, N)
    h = nat.rm_load_poles(Eg, wg, m["a"], m["e_thr"], m["l"], m["z"], 1.0)
    E = np.linspace(0.05, 3.0, 257)
    om, st = nat.rm_sweep_energies([h], 3, torch.as_tensor(E, device="cuda:0"))
    sym = {"E_pole": Eo, "w": wo, "a": m["a"], "e_thr": m["e_thr"],
           "l": m["l"], "z": m["z"], "g": 1.0}
    ref = oracle.sweep(sym, E, n_target=3)["omega"]
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref)
    log("inner -> sweep, 257 energies: Omega %.2e" % err)
    assert err < 1e-6
    h.free()


def test_argument_errors(nat):
    good = _random_model(2, 1)
    with pytest.raises(nat.RmError) as ex:
        nat.rm_inner_region(good, 8193)
    assert ex.value.code == nat.RM_ERR_ARG
    bad = dict(good, depth=np.array([[1.0, 0.2], [0.3, 1.0]]))
    with pytest.raises(nat.RmError):
        nat.rm_inner_region(bad, 8)
    bad = dict(good, range=np.array([[1.0, 0.0], [0.0, 1.0]]))
    with pytest.raises(nat.RmError):
        nat.rm_inner_region(bad, 8)
    with pytest.raises(nat.RmError):
        nat.rm_inner_region(dict(good, a=0.0), 8)
    with pytest.raises(nat.RmError):
        nat.rm_inner_region(good, 0)


def test_batch_matches_single_solves(nat):
    """Ten models (more than the 8 worker threads; D from 1 to 1024, one
    odd) through rm_inner_region_batch give bit for bit what rm_inner_region
    gives for each: the same kernels on the same inputs."""
    shapes = [(1, 1), (2, 40), (3, 15), (4, 256), (2, 64), (5, 13), (1, 300),
              (3, 100), (2, 512), (4, 32)]
    models = [_random_model(n, 40 + b) for b, (n, N) in enumerate(shapes)]
    Ns = [N for _, N in shapes]
    t0 = time.perf_counter()
    out = nat.rm_inner_region_batch(models, Ns)
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    single = [nat.rm_inner_region(m, N) for m, N in zip(models, Ns)]
    ts = time.perf_counter() - t0
    log("batch of %d: %.3f s, one by one %.3f s" % (len(models), tb, ts))
    for (Eb, wb, sb, rb), (Es, ws, ss, rs) in zip(out, single):
        assert np.array_equal(Eb, Es) and np.array_equal(wb, ws)
        assert sb == ss and rb == rs


def test_batch_reports_the_failing_item(nat):
    good = _random_model(2, 1)
    bad = dict(good, depth=np.array([[1.0, 0.2], [0.3, 1.0]]))
    with pytest.raises(nat.RmError) as ex:
        nat.rm_inner_region_batch([good, bad, good], 16)
    assert ex.value.code == nat.RM_ERR_ARG and "item 1" in str(ex.value)
    assert nat.rm_inner_region_batch([], 16) == []


@pytest.mark.parametrize("n,N,Q", [(2, 15, 45), (3, 10, 1), (1, 7, 30),
                                   (2, 9, 59)])
def test_quadrature_sizes_not_multiple_of_four(nat, n, N, Q):
    """The assembly pads the quadrature to a multiple of 4 nodes with zero
    weights: Q = 45, 1, 30, 59 give the oracle's poles and R with the same
    Q."""
    _log_and_check("n=%d N=%d Q=%d" % (n, N, Q),
                   _compare(nat, _random_model(n, 70 + Q), N, Q=Q))


@pytest.mark.parametrize("case", ["l12_small_box", "strong_charge", "large_box"])
def test_extreme_models(nat, case):
    """Models at the edges of the accepted range: l = 12 in a 3 a0 box (a
    centrifugal term of 156/r^2 dominating the spectrum), z = 5 with a deep
    well, and a 60 a0 box; the same error budget applies."""
    if case == "l12_small_box":
        m = _model([0.0, 0.5], [12, 11], 1.0, 3.0, [[3.0, 1.0], [1.0, 2.0]],
                   [[1.0, 1.5], [1.5, 1.0]])
        N = 80
    elif case == "strong_charge":
        m = _model([0.0, 0.2, 0.9], [0, 1, 2], 5.0, 10.0,
                   [[20.0, 2.0, 1.0], [2.0, 15.0, 3.0], [1.0, 3.0, 10.0]],
                   [[0.5, 1.0, 1.5], [1.0, 0.8, 1.2], [1.5, 1.2, 2.0]])
        N = 120
    else:
        m = _model([0.0, 0.1], [0, 3], 1.0, 60.0, [[2.0, 0.5], [0.5, 1.0]],
                   [[5.0, 8.0], [8.0, 6.0]])
        N = 300
    _log_and_check(case, _compare(nat, m, N))


def _invariants(nat, m, N):
    """Device solve of a large model against what the oracle's H fixes
    without its eigen-solve: by Weyl each eigenvalue is within eta, so
    sum(E) is within D eta of tr H and sum(E^2) within 2 eta sum|E| + D eta^2
    of |H|_F^2."""
    t0 = time.perf_counter()
    Eg, wg, sweeps, _ = nat.rm_inner_region(m, N)
    t_dev = time.perf_counter() - t0
    Q = N + 48
    H = inner.hamiltonian(m, N, Q)
    D = H.shape[0]
    S = max(np.abs(Eg).max(), 1.0)
    eta = 8.0 * (D + Q) * np.finfo(float).eps * S
    r_tr = abs(Eg.sum() - np.trace(H)) / (D * eta)
    r_fro = abs((Eg ** 2).sum() - (H * H).sum()) / (
        2.0 * eta * np.abs(Eg).sum() + D * eta ** 2)
    log("D=%d: device solve %.2f s, %d sweeps; trace %.2e, Frobenius %.2e of "
        "their bounds" % (D, t_dev, sweeps, r_tr, r_fro))
    assert np.all(np.diff(Eg) >= 0.0)
    assert r_tr < 1.0 and r_fro < 1.0
    return Eg, wg, H, eta


def test_dimension_8192_against_a_direct_solve(nat):
    """D = 8192: the invariants, and R(E) between the two lowest poles
    against (1/2a) B (H - E)^-1 B^T solved directly on the host, within
    (eta/2a) sqrt(G_i G_j), G_i = |(H - E)^-1 b_i|^2."""
    import scipy.linalg
    m = _random_model(4, 90)
    N = 2048
    Eg, wg, H, eta = _invariants(nat, m, N)
    n, D, a = 4, H.shape[0], m["a"]
    E = 0.5 * (Eg[0] + Eg[1])
    B = np.zeros((n, D))
    phia = np.sqrt(2.0) * np.sqrt(2.0 / a) * (-1.0) ** np.arange(N)
    for i in range(n):
        B[i, i * N:(i + 1) * N] = phia
    X = scipy.linalg.solve(H - E * np.eye(D), B.T, assume_a="sym")
    Rd = B @ X / (2.0 * a)
    Rg = (wg / (Eg - E)) @ wg.T / (2.0 * a)
    G = (X * X).sum(axis=0)
    ratio = (np.abs(Rg - Rd) / (eta / (2.0 * a) * np.sqrt(np.outer(G, G)))).max()
    log("D=8192: R between the lowest poles %.2e of its bound" % ratio)
    assert ratio < 1.0


def test_dimension_16384(nat):
    """D = 16384, the entry point's limit: the invariants, and R(E) between
    the two lowest poles against (1/2a) B (H - E)^-1 B^T, as at 8192, which
    checks the eigenvectors and surface amplitudes.  The direct solve runs
    as an FP64 LU with partial pivoting from torch's linear algebra on the
    device (a host solve of this size takes about a minute); its residual
    is checked first."""
    import torch
    m = _random_model(8, 91)
    N = 2048
    Eg, wg, H, eta = _invariants(nat, m, N)
    n, D, a = 8, H.shape[0], m["a"]
    E = 0.5 * (Eg[0] + Eg[1])
    B = np.zeros((n, D))
    phia = np.sqrt(2.0) * np.sqrt(2.0 / a) * (-1.0) ** np.arange(N)
    for i in range(n):
        B[i, i * N:(i + 1) * N] = phia
    dev = torch.device("cuda:0")
    Ht = torch.as_tensor(H, device=dev)
    Ht.diagonal().sub_(E)
    Bt = torch.as_tensor(B.T.copy(), device=dev)
    Xt = torch.linalg.solve(Ht, Bt)
    res = float((Ht @ Xt - Bt).abs().max() / (Ht.abs().sum(dim=1).max() * Xt.abs().max()))
    X = Xt.cpu().numpy()
    del Ht, Bt, Xt
    torch.cuda.empty_cache()
    assert res < 1e-12
    Rd = B @ X / (2.0 * a)
    Rg = (wg / (Eg - E)) @ wg.T / (2.0 * a)
    G = (X * X).sum(axis=0)
    ratio = (np.abs(Rg - Rd) / (eta / (2.0 * a) * np.sqrt(np.outer(G, G)))).max()
    log("D=16384: solve residual %.1e; R between the lowest poles %.2e of its "
        "bound" % (res, ratio))
    assert ratio < 1.0
