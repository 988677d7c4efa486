"""The sweep entry point that allocates nothing (rm_sweep_energies_noalloc)
against the allocating rm_sweep_energies, through the C ABI (needs an
MI355X).  Both run the same kernels on the same energies, so Omega and the
status bits must agree bit for bit; two calls in a row, the second on a
smaller input, check that nothing left in the shared scratch array from the
first call leaks into the second."""
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


def _noalloc(torch, nat, hs, n_t, E, opts=None):
    M = int(E.numel())
    P = n_t * (n_t + 1) // 2
    om = torch.full((M, P), -7.0, dtype=torch.float64, device=E.device)
    st = torch.full((M,), -1, dtype=torch.int32, device=E.device)
    nat.rm_sweep_energies_noalloc(hs, n_t, E, om, st, opts)
    torch.cuda.synchronize()
    return om.cpu().numpy(), st.cpu().numpy()


def _alloc(torch, nat, hs, n_t, E, opts=None):
    om, st = nat.rm_sweep_energies(hs, n_t, E, opts)
    torch.cuda.synchronize()
    return om.cpu().numpy(), st.cpu().numpy()


def test_noalloc_equals_sweep_c1_two_calls(env):
    """8 channels: all 2000 energies in chunks of 300 (7 chunks, ragged
    tail), then a second call on 417 energies; each equals the allocating
    sweep bit for bit, and the first matches the oracle."""
    torch, nat = env
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    opts = nat.make_opts(chunk=300)
    for count in (2000, 417):
        E = torch.as_tensor(w.mesh[:count], dtype=torch.float64,
                            device="cuda:0")
        log("noalloc c1 m=%d" % count)
        a_om, a_st = _noalloc(torch, nat, [h], 8, E, opts)
        b_om, b_st = _alloc(torch, nat, [h], 8, E, opts)
        assert np.array_equal(a_om, b_om)
        assert np.array_equal(a_st, b_st)
    ref = oracle.sweep(w.syms[0].as_dict(), w.mesh[:417])
    err, _, _ = omega_normwise_err(a_om, ref["omega"])
    assert err < 1e-6
    h.free()


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_sweep_c2_two_calls(env, prec):
    """200 channels: 700 energies (several scratch-sized chunks), then 131;
    FP64 and FP32 pole sums.  Same variants on both sides (the FP32 pair
    products are formed by the allocating call that runs first)."""
    torch, nat = env
    w = wl.config2()
    h = nat.load_symmetry(w.syms[0])
    opts = nat.make_opts(prec=prec)
    idx = np.sort(wl.sample_indices(w.mesh.size, 700, seed=21))
    for count in (700, 131):
        E = torch.as_tensor(w.mesh[idx[:count]], dtype=torch.float64,
                            device="cuda:0")
        log("noalloc c2 prec=%d m=%d" % (prec, count))
        b_om, b_st = _alloc(torch, nat, [h], 200, E, opts)
        a_om, a_st = _noalloc(torch, nat, [h], 200, E, opts)
        assert np.array_equal(a_om, b_om)
        assert np.array_equal(a_st, b_st)
    ref = oracle.sweep(w.syms[0].as_dict(), w.mesh[idx[:3]])
    err, _, _ = omega_normwise_err(a_om[:3], ref["omega"])
    log("noalloc c2 prec=%d oracle err %.2e" % (prec, err))
    assert err < (1e-6 if prec == 0 else 1e-4)
    h.free()


def test_noalloc_with_propagation_and_expansion(env):
    """c1 propagated to A = 120 and matched to the asymptotic expansion:
    the expansion's scratch comes from the same array; 600 then 250
    energies, each equal to the allocating sweep bit for bit."""
    torch, nat = env
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    rng = np.random.default_rng(1)
    beta = rng.normal(0.0, 1.0, (2, 8, 8)) * np.array([0.3, 0.6])[:, None, None]
    beta = 0.5 * (beta + beta.transpose(0, 2, 1))
    nat.rm_set_propagation(h, 120.0, 200, beta)
    nat.rm_set_gailitis(h, 40)
    opts = nat.make_opts(chunk=200)
    for count in (600, 250):
        E = torch.as_tensor(w.mesh[::3][:count], dtype=torch.float64,
                            device="cuda:0")
        log("noalloc c1 expansion m=%d" % count)
        a_om, a_st = _noalloc(torch, nat, [h], 8, E, opts)
        b_om, b_st = _alloc(torch, nat, [h], 8, E, opts)
        assert np.array_equal(a_om, b_om)
        assert np.array_equal(a_st, b_st)
        assert (a_st & nat.RM_E_ASYM_NOCONV).any()
    h.free()


def test_noalloc_rejects_autotune_and_oversized(env):
    """Autotuning (which allocates) is refused; so is a symmetry set whose
    one energy needs more than the scratch array."""
    torch, nat = env
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    E = torch.as_tensor(w.mesh[:10], dtype=torch.float64, device="cuda:0")
    om = torch.empty((10, 36), dtype=torch.float64, device="cuda:0")
    st = torch.empty((10,), dtype=torch.int32, device="cuda:0")
    with pytest.raises(nat.RmError) as ei:
        nat.rm_sweep_energies_noalloc([h], 8, E, om, st,
                                      nat.make_opts(flags=nat.RM_FLAG_AUTOTUNE))
    assert ei.value.code == nat.RM_ERR_ARG
    # 2048 channels (the handle limit): 3 n^2 doubles = 100 MB per energy,
    # three copies of the symmetry need 300 MB per energy
    rng = np.random.default_rng(3)
    big = wl.random_symmetry(rng, 2048, 64, -2.0, 40.0)
    hb = nat.load_symmetry(big)
    omb = torch.empty((10, 2048 * 2049 // 2), dtype=torch.float64,
                      device="cuda:0")
    with pytest.raises(nat.RmError) as ei:
        nat.rm_sweep_energies_noalloc([hb, hb, hb], 2048, E, omb, st)
    assert ei.value.code == nat.RM_ERR_ARG
    log("oversized: %s" % ei.value)
    hb.free()
    h.free()
