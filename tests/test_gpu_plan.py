"""Captured sweeps (rm_plan_*, hipGraph replay), batched symmetries and the
tile autotuner (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, omega_normwise_err, oracle_sweep_multi
from paper_1403_5524_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1403_5524_amd import native
    assert torch.cuda.is_available()
    return torch, native


def test_graph_replays_match_eager(env):
    """Three replays with eager work and synchronisation between them; each
    replay equals the eager sweep bit for bit (fixed reduction order)."""
    torch, nat = env
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    E = torch.as_tensor(w.mesh, dtype=torch.float64, device="cuda:0")
    ref, rst = nat.rm_sweep_energies([h], 8, E, nat.make_opts(chunk=300))
    ref = ref.cpu().numpy()
    plan = nat.Plan([h], 8, E, nat.make_opts(chunk=300))
    chunk, n_chunks, _ = plan.info()
    assert chunk == 300 and n_chunks == 7
    for rep in range(3):
        plan.omega.fill_(-1.0)
        om, st = plan.execute()
        torch.cuda.synchronize()
        assert np.array_equal(om.cpu().numpy(), ref), rep
        assert np.array_equal(st.cpu().numpy(), rst.cpu().numpy())
        nat.rm_sweep_energies([h], 8, E[:50])   # eager work in between
        torch.cuda.synchronize()
    plan.free()


def test_plan_batched_symmetries_vs_oracle(env):
    """Ten symmetries of uneven size sharing 20 target levels in one plan."""
    torch, nat = env
    w = wl.config3(M=2000)
    syms = w.syms[:10]
    hs = [nat.load_symmetry(s) for s in syms]
    idx = wl.sample_indices(w.mesh.size, 8, seed=11)
    E = torch.as_tensor(w.mesh[idx], dtype=torch.float64, device="cuda:0")
    plan = nat.Plan(hs, w.n_target, E)
    om, st = plan.execute()
    torch.cuda.synchronize()
    ref, rst = oracle_sweep_multi(syms, w.mesh[idx], w.n_target)
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref)
    log("plan batched err %.3e" % err)
    assert err < 1e-6
    assert np.array_equal(st.cpu().numpy(), rst)
    plan.free()


def test_autotuned_mixed_plan(env):
    """Autotuning picks one of the mixed variants (scaled-W tiles 1-3 or the
    pair-major GEMM 4); the result still meets the mixed tolerance."""
    torch, nat = env
    w = wl.config2(M=4096)
    h = nat.load_symmetry(w.syms[0])
    E = torch.as_tensor(w.mesh, dtype=torch.float64, device="cuda:0")
    plan = nat.Plan([h], 200, E, nat.make_opts(prec=nat.RM_PREC_BF16X3,
                                               flags=nat.RM_FLAG_AUTOTUNE))
    _, _, variants = plan.info()
    log("autotuned variant %s" % variants)
    assert variants[0] in (1, 2, 3, 4)
    om, st = plan.execute()
    torch.cuda.synchronize()
    idx = wl.sample_indices(E.numel(), 8, seed=12)
    ref = oracle.sweep(w.syms[0].as_dict(), w.mesh[idx])
    err, _, _ = omega_normwise_err(om.cpu().numpy()[idx], ref["omega"])
    assert err < 1e-4
    plan.free()
