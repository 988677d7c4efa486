"""Mixed-precision pole sums (FP32 and split-BF16 MFMA with the FP64
near-pole correction) against the FP64 oracle (needs an MI355X), for both
forms of the pole sum: the pair-major GEMM over precomputed w_ik w_jk (the
default) and the scaled-W kernels (RM_FLAG_NO_PAIR_PRODUCTS).

Bar: Omega within 1e-4 normwise per energy (the stated tolerance for the
mixed paths) at the configured near-pole window delta = 1e-3 Ry, with the
FP32-operand band out to 1e-2 Ry (the defaults).  R is checked normwise
against bounds that follow from the arithmetic: FP32 operands carry 24
bits, split BF16 about 16 bits, with FP32 accumulation over N_H terms.
The elementwise error (every transition at least 1e-8 of its row's
largest) is logged, not asserted: weak transitions carry the absolute
error of the strong ones.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, omega_elementwise_err, omega_normwise_err
from paper_1403_5524_amd import workloads as wl

pytestmark = pytest.mark.gpu

OMEGA_TOL_MIXED = 1e-4
DELTA = 1e-3   # the configured near-pole window of the 200-channel case
R_TOL = {1: 1e-5, 2: 1e-4}
FORMS = [0, 0x2]   # pair-major GEMM, scaled-W kernels


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1403_5524_amd import native
    assert torch.cuda.is_available()
    w = wl.config2()
    h = native.load_symmetry(w.syms[0])
    return torch, native, w, h


def _near_pole_energies(sym, count, offset):
    """Energies offset Ry from poles inside [0.5, 19.5]."""
    ks = np.nonzero((sym.E_pole > 0.5) & (sym.E_pole < 19.5))[0]
    pick = ks[np.linspace(0, ks.size - 1, count).astype(int)]
    return sym.E_pole[pick] + offset


@pytest.mark.parametrize("flags", FORMS)
@pytest.mark.parametrize("prec", [1, 2])
def test_rmatrix_mixed_c2(env, prec, flags):
    torch, nat, w, h = env
    s = w.syms[0]
    E = np.concatenate([w.mesh[wl.sample_indices(w.mesh.size, 12, seed=8)],
                        _near_pole_energies(s, 4, 1e-6),
                        _near_pole_energies(s, 4, -3e-4)])
    log("rmatrix mixed prec=%d flags=%d m=%d" % (prec, flags, E.size))
    Et = torch.as_tensor(E, dtype=torch.float64, device="cuda:0")
    R = nat.rm_rmatrix(h, Et, nat.make_opts(prec=prec, flags=flags)).cpu().numpy()
    Rr = oracle.r_matrix(s.E_pole, s.w, s.a, E)
    err = np.abs(R - Rr).max(axis=(1, 2)) / np.abs(Rr).max(axis=(1, 2))
    log("R normwise err max %.3e" % err.max())
    assert err.max() < R_TOL[prec]


def _tier_energies(sym, w):
    """Mesh energies plus energies in every tier of the pole sum around a
    pole: inside the FP64 window (2e-6), just outside it and across the
    FP32-operand band (1.05e-3 ... 9e-3, both sides), and just beyond the
    band (1.2e-2, 1.5e-2), where the far sum carries its largest terms."""
    rng = np.random.default_rng(17)
    ks = np.nonzero((sym.E_pole > 0.5) & (sym.E_pole < 19.5))[0]
    pk = rng.choice(ks, 40, replace=False)
    off = rng.uniform(1.0e-3, 5.0e-3, 40) * rng.choice([-1.0, 1.0], 40)
    off[:8] = np.sign(off[:8]) * rng.uniform(1.0e-3, 1.1e-3, 8)
    return np.concatenate([w.mesh[wl.sample_indices(w.mesh.size, 24, seed=9)],
                           sym.E_pole[pk] + off,
                           _near_pole_energies(sym, 4, 2e-6),
                           _near_pole_energies(sym, 4, 9e-3),
                           _near_pole_energies(sym, 4, -1.05e-3),
                           _near_pole_energies(sym, 4, 1.2e-2),
                           _near_pole_energies(sym, 4, -1.5e-2)])


@pytest.fixture(scope="module")
def tier_ref(env):
    _, _, w, _ = env
    s = w.syms[0]
    E = _tier_energies(s, w)
    return E, oracle.sweep(s.as_dict(), E)


@pytest.mark.parametrize("flags", FORMS)
@pytest.mark.parametrize("prec", [1, 2])
def test_sweep_mixed_c2_delta_1e3(env, tier_ref, prec, flags):
    """The 200-channel case at delta = 1e-3 Ry (its configuration): 24 mesh
    energies and 60 energies placed in every tier around poles, half of
    them 1-5e-3 Ry from a pole."""
    torch, nat, w, h = env
    E, ref = tier_ref
    log("sweep mixed prec=%d flags=%d m=%d delta=%g" % (prec, flags, E.size,
                                                         DELTA))
    Et = torch.as_tensor(E, dtype=torch.float64, device="cuda:0")
    om, st = nat.rm_sweep_energies([h], 200, Et,
                                   nat.make_opts(prec=prec, flags=flags,
                                                 near_delta=DELTA))
    om = om.cpu().numpy()
    err, _, _ = omega_normwise_err(om, ref["omega"])
    el = omega_elementwise_err(om, ref["omega"])
    log("mixed prec=%d flags=%d omega normwise err %.3e (elementwise %.3e)"
        % (prec, flags, err, el))
    assert err < OMEGA_TOL_MIXED
    assert np.array_equal(st.cpu().numpy(), ref["status"])


def test_default_window_is_the_configured_one(env, tier_ref):
    """A zero-initialised rm_opts selects delta = 1e-3 and the band edge
    10 delta: bit-identical to asking for them."""
    torch, nat, w, h = env
    E, _ = tier_ref
    Et = torch.as_tensor(E[:16], dtype=torch.float64, device="cuda:0")
    a, _ = nat.rm_sweep_energies([h], 200, Et, nat.make_opts(prec=1))
    b, _ = nat.rm_sweep_energies([h], 200, Et,
                                 nat.make_opts(prec=1, near_delta=1e-3,
                                               band_delta=1e-2))
    assert torch.equal(a, b)


def test_band_is_what_meets_the_tolerance(env, tier_ref):
    """With the band switched off (band_delta = delta) the FP32-accumulated
    far sum carries the poles 1-5e-3 Ry away and misses the tolerance that
    the three-tier sum meets: the band is doing the work."""
    torch, nat, w, h = env
    E, ref = tier_ref
    Et = torch.as_tensor(E, dtype=torch.float64, device="cuda:0")
    om, _ = nat.rm_sweep_energies([h], 200, Et,
                                  nat.make_opts(prec=1, near_delta=DELTA,
                                                band_delta=DELTA))
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref["omega"])
    log("fp32 without the band: omega normwise err %.3e" % err)
    assert err > OMEGA_TOL_MIXED


def test_mixed_matches_fp64_on_c1(env):
    """Small system: every energy of the 8-channel case (one padded pair
    block, 16 energy blocks with a ragged last one), both mixed paths and
    both forms."""
    torch, nat, _, _ = env
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    Et = torch.as_tensor(w.mesh, dtype=torch.float64, device="cuda:0")
    ref = oracle.sweep(w.syms[0].as_dict(), w.mesh)
    for prec in (1, 2):
        for flags in FORMS:
            om, _ = nat.rm_sweep_energies([h], 8, Et,
                                          nat.make_opts(prec=prec, flags=flags))
            err, _, _ = omega_normwise_err(om.cpu().numpy(), ref["omega"])
            log("c1 mixed prec=%d flags=%d err %.3e" % (prec, flags, err))
            assert err < OMEGA_TOL_MIXED


def test_pair_form_matches_scaled_w_form(env):
    """The two forms of the mixed pole sum agree on R to the precision of
    their operands (both round the same FP64 products and reciprocals)."""
    torch, nat, w, h = env
    E = w.mesh[wl.sample_indices(w.mesh.size, 300, seed=11)]
    Et = torch.as_tensor(E, dtype=torch.float64, device="cuda:0")
    for prec in (1, 2):
        Ra = nat.rm_rmatrix(h, Et, nat.make_opts(prec=prec)).cpu().numpy()
        Rb = nat.rm_rmatrix(h, Et, nat.make_opts(prec=prec, flags=0x2)).cpu().numpy()
        d = np.abs(Ra - Rb).max(axis=(1, 2)) / np.abs(Rb).max(axis=(1, 2))
        log("pair vs scaled-W prec=%d max normwise diff %.3e" % (prec, d.max()))
        assert d.max() < 2 * R_TOL[prec]
        assert np.array_equal(Ra, Ra.transpose(0, 2, 1))
