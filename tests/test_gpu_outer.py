"""Outer-region propagation through the C ABI vs the FP64 oracle (needs an
MI355X).  Both sides use the same sectors, so they agree to rounding: K
within 1e-8 of max(1, |K|), Omega within 1e-6 normwise (the path's FP64
bound).  The pure-Coulomb case compares with matching at r = a, up to the
second-order sector error."""
import numpy as np
import pytest

import oracle
from oracle import outer
from gpu_helpers import log, omega_normwise_err
from paper_1403_5524_amd import workloads as wl

pytestmark = pytest.mark.gpu


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


def _beta(n, seed, scales=(1.5, 6.0)):
    rng = np.random.default_rng(seed)
    out = []
    for sc in scales:
        M = rng.normal(0.0, sc, (n, n))
        out.append(0.5 * (M + M.T))
    return np.stack(out)


def _dev(torch, dev, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                           device=dev)


def _k_err(nat, torch, dev, h, sym, prop, E):
    K, no, _, st = nat.rm_kmatrix(h, _dev(torch, dev, E))
    K, no = K.cpu().numpy(), no.cpu().numpy()
    worst = 0.0
    for m, Ee in enumerate(E):
        Kr, P = outer.k_matrix_propagated(sym, prop, Ee)
        assert no[m] == P.size
        if P.size == 0:
            continue
        Kg = K[m, :P.size, :P.size]
        worst = max(worst, np.abs(Kg - Kr).max() / max(1.0, np.abs(Kr).max()))
    return worst, st.cpu().numpy()


def test_kmatrix_with_multipole_coupling(torch_dev, nat):
    torch, dev = torch_dev
    w = wl.config1()
    sym = w.syms[0].as_dict()
    h = nat.load_symmetry(w.syms[0])
    prop = {"A": sym["a"] + 10.0, "n_sec": 20, "beta": _beta(8, 1)}
    nat.rm_set_propagation(h, prop["A"], prop["n_sec"], prop["beta"])
    E = w.mesh[::37]
    err, st = _k_err(nat, torch, dev, h, sym, prop, E)
    log("propagated K, %d energies: %.2e" % (E.size, err))
    assert err < 1e-8
    h.free()


def test_sweep_with_multipole_coupling(torch_dev, nat):
    torch, dev = torch_dev
    w = wl.config1()
    sym = w.syms[0].as_dict()
    h = nat.load_symmetry(w.syms[0])
    prop = {"A": sym["a"] + 12.0, "n_sec": 16, "beta": _beta(8, 2)}
    nat.rm_set_propagation(h, prop["A"], prop["n_sec"], prop["beta"])
    E = w.mesh[::13]
    om, st = nat.rm_sweep_energies([h], 8, _dev(torch, dev, E),
                                   nat.make_opts(chunk=37))
    ref = outer.sweep_propagated(sym, prop, E, n_target=8)
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref)
    log("propagated Omega, %d energies: %.2e" % (E.size, err))
    assert err < 1e-6
    h.free()


def test_pure_coulomb_outer_region_and_switch_off(torch_dev, nat):
    """No multipoles: K after propagating to A equals K matched at a up to
    the sector error; n_sec = 0 restores the unpropagated K bit for bit."""
    torch, dev = torch_dev
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    E = _dev(torch, dev, w.mesh[500::150])
    K0, no0, _, _ = nat.rm_kmatrix(h, E)
    nat.rm_set_propagation(h, w.syms[0].a + 15.0, 600)
    K1, no1, _, _ = nat.rm_kmatrix(h, E)
    assert np.array_equal(no0.cpu().numpy(), no1.cpu().numpy())
    d = (K1 - K0).abs().max().item() / max(1.0, K0.abs().max().item())
    log("pure Coulomb propagation vs matching at a: %.2e" % d)
    assert d < 1e-4
    nat.rm_set_propagation(h, 0.0, 0)
    K2, _, _, _ = nat.rm_kmatrix(h, E)
    assert torch.equal(K2, K0)
    h.free()


def test_kmatrix_200_channels_sampled(torch_dev, nat):
    torch, dev = torch_dev
    w = wl.config2()
    sym = w.syms[0].as_dict()
    h = nat.load_symmetry(w.syms[0])
    prop = {"A": sym["a"] + 6.0, "n_sec": 12, "beta": _beta(200, 3, (0.5, 2.0))}
    nat.rm_set_propagation(h, prop["A"], prop["n_sec"], prop["beta"])
    idx = wl.sample_indices(w.mesh.size, 6, seed=8)
    err, st = _k_err(nat, torch, dev, h, sym, prop, w.mesh[idx])
    log("propagated K, 200 channels: %.2e" % err)
    assert err < 1e-8
    h.free()
