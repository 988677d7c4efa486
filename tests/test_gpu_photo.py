"""Photoionization through the C ABI vs the FP64 oracle (needs an MI355X).

Tolerance: sigma of the FP64 path within 1e-6 of the oracle relative to the
largest reference value on the mesh (the same bound as Omega: sigma is a
quadratic form of the same solution); mixed-precision R pole sums within
1e-4 on the same measure.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import log
from paper_1403_5524_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-6
TOL_MIXED = 1e-4
E0 = -0.8   # initial state below every threshold


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


def _dip(sym, seed):
    return np.random.default_rng(seed).normal(size=sym.n_poles)


def _err(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def c1(nat):
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    d = _dip(w.syms[0], 11)
    nat.rm_load_dipoles(h, d)
    return w, h, d


def test_photo_small_full_mesh(torch_dev, nat, c1):
    """8 channels, 200 poles, all 2000 energies of [0, 10] (open and closed
    channels, a ragged last matching chunk)."""
    torch, dev = torch_dev
    w, h, d = c1
    E = torch.as_tensor(w.mesh, dtype=torch.float64, device=dev)
    opts = nat.make_opts(chunk=384)
    sig, st = nat.rm_photoionization([h], E, E0, opts)
    ref = oracle.photoionization([w.syms[0].as_dict()], [d], w.mesh, E0)
    err = _err(sig.cpu().numpy(), ref)
    st = st.cpu().numpy()
    log("photo c1: max error %.2e, flagged %d" % (err, int((st != 0).sum())))
    below = w.mesh <= w.syms[0].e_thr.min()
    assert np.all(sig.cpu().numpy()[below] == 0.0)
    assert np.all((st[below] & nat.RM_E_NO_OPEN) != 0)
    assert np.all(st[~below] == 0)
    assert err < TOL_FP64


def test_photo_two_symmetries_add(torch_dev, nat, c1):
    torch, dev = torch_dev
    w, h, d = c1
    w2 = wl.single(6, 150, -1.0, 40.0, 0.0, 10.0, 300, 21, "aux")
    h2 = nat.load_symmetry(w2.syms[0])
    d2 = _dip(w2.syms[0], 12)
    nat.rm_load_dipoles(h2, d2)
    Em = w.mesh[::7]
    E = torch.as_tensor(Em, dtype=torch.float64, device=dev)
    sig, _ = nat.rm_photoionization([h, h2], E, E0)
    ref = oracle.photoionization([w.syms[0].as_dict(), w2.syms[0].as_dict()],
                                 [d, d2], Em, E0)
    err = _err(sig.cpu().numpy(), ref)
    log("photo two symmetries: %.2e" % err)
    assert err < TOL_FP64
    h2.free()


@pytest.mark.parametrize("prec", [1, 2])
def test_photo_mixed_pole_sum(torch_dev, nat, c1, prec):
    torch, dev = torch_dev
    w, h, d = c1
    Em = w.mesh[::5]
    E = torch.as_tensor(Em, dtype=torch.float64, device=dev)
    sig, _ = nat.rm_photoionization([h], E, E0, nat.make_opts(prec=prec))
    ref = oracle.photoionization([w.syms[0].as_dict()], [d], Em, E0)
    err = _err(sig.cpu().numpy(), ref)
    log("photo prec %d: %.2e" % (prec, err))
    assert err < TOL_MIXED


def test_photo_requires_dipoles(torch_dev, nat):
    torch, dev = torch_dev
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    E = torch.as_tensor(w.mesh[:8], dtype=torch.float64, device=dev)
    with pytest.raises(nat.RmError) as ei:
        nat.rm_photoionization([h], E, E0)
    assert ei.value.code == nat.RM_ERR_ARG
    h.free()


def test_photo_200_channels_sampled(torch_dev, nat):
    """The 200-channel, 8000-pole symmetry over its whole 1e5-point mesh on
    the GPU; 12 sampled energies against the oracle."""
    torch, dev = torch_dev
    w = wl.config2()
    h = nat.load_symmetry(w.syms[0])
    d = _dip(w.syms[0], 13)
    nat.rm_load_dipoles(h, d)
    E = torch.as_tensor(w.mesh, dtype=torch.float64, device=dev)
    sig, st = nat.rm_photoionization([h], E, E0)
    torch.cuda.synchronize()
    idx = wl.sample_indices(w.mesh.size, 12, seed=5)
    ref = oracle.photoionization([w.syms[0].as_dict()], [d], w.mesh[idx], E0)
    got = sig.cpu().numpy()[idx]
    err = _err(got, ref)
    log("photo c2 sampled: %.2e" % err)
    assert err < TOL_FP64
    assert np.all(np.isfinite(sig.cpu().numpy()))
    h.free()


def test_photo_b2_shape_sampled(torch_dev, nat):
    """The B II photoionization shape (400 channels, 24,800 poles): 512
    energies spread over its 409,600-point mesh on the GPU, 4 of them against
    the oracle."""
    torch, dev = torch_dev
    w, d, e0 = wl.photo_b2()
    h = nat.load_symmetry(w.syms[0])
    nat.rm_load_dipoles(h, d)
    Em = w.mesh[::800]
    E = torch.as_tensor(Em, dtype=torch.float64, device=dev)
    sig, st = nat.rm_photoionization([h], E, e0)
    torch.cuda.synchronize()
    idx = wl.sample_indices(Em.size, 4, seed=3)
    ref = oracle.photoionization([w.syms[0].as_dict()], [d], Em[idx], e0)
    err = _err(sig.cpu().numpy()[idx], ref)
    log("photo b2 sampled: %.2e" % err)
    assert err < TOL_FP64
    h.free()


def test_photo_ca2_shape_sampled(torch_dev, nat):
    """The Ca II photoionization shape of Table 2 (1815 channels, 23,073
    poles): 250 energies spread over its 6000-point mesh in one chunk on the
    GPU, 2 of them against the oracle."""
    torch, dev = torch_dev
    w, d, e0 = wl.photo_ca2()
    h = nat.load_symmetry(w.syms[0])
    nat.rm_load_dipoles(h, d)
    Em = w.mesh[::24]
    E = torch.as_tensor(Em, dtype=torch.float64, device=dev)
    sig, st = nat.rm_photoionization([h], E, e0)
    torch.cuda.synchronize()
    idx = wl.sample_indices(Em.size, 2, seed=3)
    ref = oracle.photoionization([w.syms[0].as_dict()], [d], Em[idx], e0)
    err = _err(sig.cpu().numpy()[idx], ref)
    log("photo ca2 sampled: %.2e" % err)
    assert err < TOL_FP64
    h.free()


# ---- radiation damping -----------------------------------------------------

def _damped_opts(nat, **kw):
    return nat.make_opts(flags=nat.RM_FLAG_RADIATION_DAMPING, **kw)


def test_photo_damped_small_full_mesh(torch_dev, nat, c1):
    """8 channels, 200 poles with radiative widths 1e-6 - 1e-3 Ry, all 2000
    energies (open and closed channels, ragged chunks): the damped cross
    section against the oracle's driven solution; below every threshold 0
    with RM_E_NO_OPEN."""
    torch, dev = torch_dev
    w, h, d = c1
    G = wl.radiative_widths(w.syms[0].n_poles, 61)
    nat.rm_load_widths(h, G)
    E = torch.as_tensor(w.mesh, dtype=torch.float64, device=dev)
    sig, st = nat.rm_photoionization([h], E, E0, _damped_opts(nat, chunk=384))
    sig, st = sig.cpu().numpy(), st.cpu().numpy()
    ref = oracle.photoionization_damped([w.syms[0].as_dict()], [d], [G],
                                        w.mesh, E0)
    err = _err(sig, ref)
    log("damped photo c1: max error %.2e" % err)
    below = w.mesh <= w.syms[0].e_thr.min()
    assert np.all(sig[below] == 0.0)
    assert np.all((st[below] & nat.RM_E_NO_OPEN) != 0)
    assert np.all(st[~below] == 0)
    assert err < TOL_FP64
    # damping only removes flux near resonances: the damped cross section
    # differs from the undamped one, by far more than the tolerance
    und = oracle.photoionization([w.syms[0].as_dict()], [d], w.mesh, E0)
    assert _err(sig, und) > 100 * TOL_FP64


def test_photo_damped_zero_widths_is_undamped(torch_dev, nat, c1):
    """With every width 0 the damped path (complex driven system) equals the
    undamped one (K-matrix route) to rounding."""
    torch, dev = torch_dev
    w, h, d = c1
    nat.rm_load_widths(h, np.zeros(w.syms[0].n_poles))
    Em = w.mesh[::5]
    E = torch.as_tensor(Em, dtype=torch.float64, device=dev)
    a, _ = nat.rm_photoionization([h], E, E0, _damped_opts(nat))
    b, _ = nat.rm_photoionization([h], E, E0)
    err = _err(a.cpu().numpy(), b.cpu().numpy())
    log("damped with zero widths vs undamped: %.2e" % err)
    assert err < 1e-10


def test_photo_damped_two_symmetries_add(torch_dev, nat, c1):
    torch, dev = torch_dev
    w, h, d = c1
    G = wl.radiative_widths(w.syms[0].n_poles, 62)
    nat.rm_load_widths(h, G)
    w2 = wl.single(6, 150, -1.0, 40.0, 0.0, 10.0, 300, 21, "aux")
    h2 = nat.load_symmetry(w2.syms[0])
    d2 = _dip(w2.syms[0], 12)
    G2 = wl.radiative_widths(w2.syms[0].n_poles, 63)
    nat.rm_load_dipoles(h2, d2)
    nat.rm_load_widths(h2, G2)
    Em = w.mesh[::7]
    E = torch.as_tensor(Em, dtype=torch.float64, device=dev)
    sig, _ = nat.rm_photoionization([h, h2], E, E0, _damped_opts(nat))
    ref = oracle.photoionization_damped(
        [w.syms[0].as_dict(), w2.syms[0].as_dict()], [d, d2], [G, G2], Em, E0)
    err = _err(sig.cpu().numpy(), ref)
    log("damped photo, two symmetries: %.2e" % err)
    assert err < TOL_FP64
    h2.free()


def test_photo_damped_b2_shape_sampled(torch_dev, nat):
    """The B II shape of the paper's Table 1 (400 channels, 24,800 poles)
    damped: 512 of its energies through the device, 3 against the oracle."""
    torch, dev = torch_dev
    w, d, e0 = wl.photo_b2()
    G = wl.radiative_widths(w.syms[0].n_poles, 65)
    h = nat.load_symmetry(w.syms[0])
    nat.rm_load_dipoles(h, d)
    nat.rm_load_widths(h, G)
    Em = w.mesh[::800][:512]
    E = torch.as_tensor(Em, dtype=torch.float64, device=dev)
    sig, st = nat.rm_photoionization([h], E, e0, _damped_opts(nat))
    idx = wl.sample_indices(Em.size, 3, seed=9)
    ref = oracle.photoionization_damped([w.syms[0].as_dict()], [d], [G],
                                        Em[idx], e0)
    err = _err(sig.cpu().numpy()[idx], ref)
    log("damped photo b2: %.2e on %d energies" % (err, idx.size))
    assert err < TOL_FP64
    h.free()


def test_photo_damped_rejects_missing_widths(torch_dev, nat):
    torch, dev = torch_dev
    w = wl.tiny()
    h = nat.load_symmetry(w.syms[0])
    nat.rm_load_dipoles(h, _dip(w.syms[0], 3))
    E = torch.as_tensor(w.mesh[:4], dtype=torch.float64, device=dev)
    with pytest.raises(nat.RmError) as ei:
        nat.rm_photoionization([h], E, E0, _damped_opts(nat))
    assert ei.value.code == nat.RM_ERR_ARG
    h.free()
