"""The matching solve factored in FP32 and refined in FP64 (rm_opts
solve_fp32 = 1) against the FP64 oracle (needs an MI355X).

Refinement runs until the FP64 residual of the matching system passes the
dsgesv-style test, so with the FP64 pole sum the result must meet the FP64
tolerance (1e-6 on Omega); with mixed pole sums, the mixed one (1e-4).  The
40000-pole, 1500-channel case runs in its configured arithmetic: split-BF16
pole sum, FP32 factorisation with FP64 refinement.  Energies a few 1e-9 Ry
from a pole make the division-free system ill-conditioned (R holds one
term of size w^2/(2a)/1e-9): there refinement may not converge, and such an
energy must then carry RM_E_REFINE_NOCONV and is solved again with the FP64
factorisation, so every energy meets the tolerance; status bits other
than that one equal the oracle's."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, omega_normwise_err
from paper_1403_5524_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1403_5524_amd import native
    assert torch.cuda.is_available()
    return torch, native


def _E(torch, x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda:0")


def test_fp32_solve_c1_every_energy(env):
    torch, nat = env
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    ref = oracle.sweep(w.syms[0].as_dict(), w.mesh)
    om, st = nat.rm_sweep_energies([h], 8, _E(torch, w.mesh),
                                   nat.make_opts(solve_fp32=1))
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref["omega"])
    st = st.cpu().numpy()
    log("c1 fp32 solve: omega err %.3e, %d energies flagged"
        % (err, int((st & nat.RM_E_REFINE_NOCONV).sum() > 0)))
    assert err < 1e-6
    assert np.array_equal(st, ref["status"])
    h.free()


@pytest.fixture(scope="module")
def c2(env):
    torch, nat = env
    w = wl.config2()
    s = w.syms[0]
    rng = np.random.default_rng(23)
    ks = np.nonzero((s.E_pole > 0.5) & (s.E_pole < 19.5))[0]
    near = s.E_pole[rng.choice(ks, 12, replace=False)] + \
        rng.choice([-1.0, 1.0], 12) * np.array([1e-6] * 4 + [1e-4] * 4 + [3e-3] * 4)
    E = np.concatenate([w.mesh[wl.sample_indices(w.mesh.size, 12, seed=31)],
                        near])
    return nat.load_symmetry(s), s, E, oracle.sweep(s.as_dict(), E)


@pytest.mark.parametrize("prec,tol", [(0, 1e-6), (1, 1e-4), (2, 1e-4)])
def test_fp32_solve_c2_sample(env, c2, prec, tol):
    """200 channels: mesh energies and energies 1e-6, 1e-4 and 3e-3 Ry from
    poles; with the FP64 pole sum within the FP64 tolerance, with FP32 and
    split-BF16 pole sums within the mixed one."""
    torch, nat = env
    h, s, E, ref = c2
    om, st = nat.rm_sweep_energies([h], 200, _E(torch, E),
                                   nat.make_opts(prec=prec, solve_fp32=1))
    err, num, den = omega_normwise_err(om.cpu().numpy(), ref["omega"])
    log("c2 fp32 solve prec=%d: omega err %.3e; per energy %s; status %s"
        % (prec, err, np.array2string(num / den, precision=1),
           st.cpu().numpy()))
    assert err < tol
    st = st.cpu().numpy()
    assert np.array_equal(st & ~nat.RM_E_REFINE_NOCONV, ref["status"])


def test_fp32_solve_kmatrix_equals_fp64_solve(env, c2):
    """K from the refined FP32 solve against K from the FP64 LU (both FP64
    pole sums): the refinement reaches the FP64 solution to the
    conditioning of the system."""
    torch, nat = env
    h, s, E, _ = c2
    Et = _E(torch, E)
    K64, no, _, st64 = nat.rm_kmatrix(h, Et)
    K32, no32, _, st32 = nat.rm_kmatrix(h, Et, nat.make_opts(solve_fp32=1))
    K64, K32 = K64.cpu().numpy(), K32.cpu().numpy()
    assert np.array_equal(no.cpu().numpy(), no32.cpu().numpy())
    d = np.abs(K32 - K64).max(axis=(1, 2)) / np.maximum(
        np.abs(K64).max(axis=(1, 2)), 1.0)
    log("fp32-solve K vs fp64-solve K: max normwise diff %.3e" % d.max())
    assert d.max() < 1e-9


def test_fp32_solve_flags_what_it_cannot_refine(env):
    """Energies 2e-9 Ry from a pole: the FP32 factors of a system with one
    term of R near 1e5 cannot reach the FP64 residual in one correction, so
    with refine_iters = 1 every such energy is flagged, and solved again in
    FP64: Omega stays within the FP64 tolerance either way."""
    torch, nat = env
    w = wl.config1()
    s = w.syms[0]
    h = nat.load_symmetry(s)
    ks = np.nonzero((s.E_pole > 2.5) & (s.E_pole < 9.5))[0][:6]
    E = s.E_pole[ks] + 2e-9
    ref = oracle.sweep(s.as_dict(), E)
    Et = _E(torch, E)
    for iters in (1, 0):
        om, st = nat.rm_sweep_energies([h], 8, Et,
                                       nat.make_opts(solve_fp32=1,
                                                     refine_iters=iters))
        om, st = om.cpu().numpy(), st.cpu().numpy()
        err, _, _ = omega_normwise_err(om, ref["omega"])
        log("refine_iters=%d at 2e-9 Ry from poles: status %s, err %.2e"
            % (iters, st, err))
        if iters == 1:
            assert (st & nat.RM_E_REFINE_NOCONV).all()
        assert err < 1e-6
        assert np.array_equal(st & ~nat.RM_E_REFINE_NOCONV, ref["status"])
    h.free()


def test_fp32_solve_c4_configured_path(env):
    """1500 channels, 40000 poles in the arithmetic the case names: split-
    BF16 pole sum, FP32 factorisation with FP64 refinement, on 2 sampled
    energies of its mesh."""
    torch, nat = env
    w = wl.config4()
    s = w.syms[0]
    h = nat.load_symmetry(s)
    E = w.mesh[wl.sample_indices(w.mesh.size, 2, seed=41)]
    ref = oracle.sweep(s.as_dict(), E)
    om, st = nat.rm_sweep_energies([h], 1500, _E(torch, E),
                                   nat.make_opts(prec=nat.RM_PREC_BF16X3,
                                                 solve_fp32=1))
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref["omega"])
    log("c4 bf16x3 + fp32 solve: omega err %.3e" % err)
    assert err < 1e-4
    assert np.array_equal(st.cpu().numpy(), ref["status"])
    h.free()
