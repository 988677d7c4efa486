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


_TUNE_SCRIPT = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_1403_5524_amd import native as nat, workloads as wl
w = wl.config1()
h = nat.load_symmetry(w.syms[0])
E = torch.as_tensor(w.mesh[:256], dtype=torch.float64, device="cuda:0")
# FP64 with autotuning: must keep the file's valid mixed entry
o64, _ = nat.rm_sweep_energies([h], 8, E, nat.make_opts(flags=nat.RM_FLAG_AUTOTUNE))
# mixed: the file's FP64-only variant for this class must be ignored
omx, _ = nat.rm_sweep_energies([h], 8, E, nat.make_opts(prec=1))
torch.cuda.synchronize()
np.save(sys.argv[2], np.stack([o64.cpu().numpy(), omx.cpu().numpy()]))
"""


def test_tune_cache_file_is_validated_and_kept(env, tmp_path):
    """RM_TUNE_CACHE: an entry whose variant belongs to another precision
    (a mixed class pointing at the FP64 pair kernel) is ignored, and an FP64
    autotune run rewrites the file without dropping the mixed entries read
    from it.  Run in a child process: the file is read once per process."""
    import os
    import subprocess
    import sys
    torch, nat = env
    cache = tmp_path / "tune.txt"
    # 8 channels, 200 poles: prec 1 -> PS_PD64 (wrong precision), and a
    # valid mixed entry for another class that must survive
    cache.write_text("8 200 1 5\n77 999 2 3\n")
    out = tmp_path / "om.npy"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env_vars = dict(os.environ, RM_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", _TUNE_SCRIPT, root, str(out)],
                       env=env_vars, capture_output=True, text=True,
                       timeout=300)
    log(r.stdout[-2000:] + r.stderr[-2000:])
    assert r.returncode == 0
    om = np.load(out)
    w = wl.config1()
    ref = oracle.sweep(w.syms[0].as_dict(), w.mesh[:256])["omega"]
    err64, _, _ = omega_normwise_err(om[0], ref)
    errmx, _, _ = omega_normwise_err(om[1], ref)
    log("tune cache: fp64 err %.2e, fp32 err %.2e" % (err64, errmx))
    assert err64 < 1e-6 and errmx < 1e-4
    lines = cache.read_text().split("\n")
    assert "77 999 2 3" in lines
    assert "8 200 1 5" not in lines
