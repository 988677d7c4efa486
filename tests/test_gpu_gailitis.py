"""Matching at A to the coupled asymptotic expansion (rm_set_gailitis)
through the C ABI against the FP64 oracle (needs an MI355X).  Both sides sum
the same terms (the smallest-term truncation decides alike), so they agree
to rounding: K within 1e-8 of max(1, |K|), Omega within 1e-6 normwise, and
the energies flagged RM_E_ASYM_NOCONV are those the oracle flags."""
import numpy as np
import pytest

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


def _beta(n, seed, scales):
    rng = np.random.default_rng(seed)
    out = []
    for sc in scales:
        M = rng.normal(0.0, sc, (n, n))
        out.append(0.5 * (M + M.T))
    return np.stack(out)


def _dev(torch, dev, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                           device=dev)


def test_sweep_with_expansion_c1(torch_dev, nat):
    """8 channels, propagated to A = 120 through 200 sectors, expansion of
    up to 40 terms: Omega and the non-convergence flags."""
    torch, dev = torch_dev
    w = wl.config1()
    sym = w.syms[0].as_dict()
    h = nat.load_symmetry(w.syms[0])
    prop = {"A": 120.0, "n_sec": 200, "beta": _beta(8, 1, (0.3, 0.6)),
            "gailitis_terms": 40}
    nat.rm_set_propagation(h, prop["A"], prop["n_sec"], prop["beta"])
    nat.rm_set_gailitis(h, prop["gailitis_terms"])
    E = w.mesh[::29]
    om, st = nat.rm_sweep_energies([h], 8, _dev(torch, dev, E),
                                   nat.make_opts(chunk=61))
    ref, flags = outer.sweep_propagated_gailitis(sym, prop, E, n_target=8)
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref)
    got = (st.cpu().numpy() & nat.RM_E_ASYM_NOCONV) != 0
    log("expansion Omega, %d energies: %.2e; flagged %d (oracle %d)"
        % (E.size, err, int(got.sum()), int(flags.sum())))
    assert err < 1e-6
    assert np.array_equal(got, flags)
    assert 0 < flags.sum() < E.size  # both kinds of energy are covered
    h.free()


def test_kmatrix_200_channels_expansion_sampled(torch_dev, nat):
    """The 200-channel symmetry (degenerate channel groups, dipole coupling
    inside them) at sampled mesh energies: more than one column block."""
    torch, dev = torch_dev
    w = wl.config2()
    sym = w.syms[0].as_dict()
    h = nat.load_symmetry(w.syms[0])
    prop = {"A": sym["a"] + 60.0, "n_sec": 60,
            "beta": _beta(200, 3, (0.5, 2.0)), "gailitis_terms": 30}
    nat.rm_set_propagation(h, prop["A"], prop["n_sec"], prop["beta"])
    nat.rm_set_gailitis(h, prop["gailitis_terms"])
    idx = wl.sample_indices(w.mesh.size, 4, seed=8)
    E = w.mesh[idx]
    K, no, _, st = nat.rm_kmatrix(h, _dev(torch, dev, E))
    K, no, st = K.cpu().numpy(), no.cpu().numpy(), st.cpu().numpy()
    worst = 0.0
    for m, Ee in enumerate(E):
        Kr, P, fl = outer.k_matrix_propagated_gailitis(sym, prop, Ee)
        assert no[m] == P.size
        assert bool(st[m] & nat.RM_E_ASYM_NOCONV) == fl
        if P.size == 0:
            continue
        Kg = K[m, :P.size, :P.size]
        worst = max(worst, np.abs(Kg - Kr).max() / max(1.0, np.abs(Kr).max()))
    log("expansion K, 200 channels, open %s: %.2e" % (no.tolist(), worst))
    assert worst < 1e-8
    h.free()


def test_expansion_without_coupling_and_switches(torch_dev, nat):
    """No multipoles and A far out: the expansion is the Coulomb function,
    so K equals the Coulomb matching at A; max_terms = 0 restores that K bit
    for bit; the expansion needs the propagation; the FP32 solve refuses
    it."""
    torch, dev = torch_dev
    w = wl.config1()
    h = nat.load_symmetry(w.syms[0])
    E = _dev(torch, dev, w.mesh[700::130])  # 3.5 Ry and up
    with pytest.raises(nat.RmError) as ex:
        nat.rm_set_gailitis(h, 20)
    assert ex.value.code == nat.RM_ERR_STATE
    nat.rm_set_propagation(h, 400.0, 400)
    K0, _, _, _ = nat.rm_kmatrix(h, E)
    nat.rm_set_gailitis(h, 60)
    K1, _, _, st = nat.rm_kmatrix(h, E)
    assert not (st.cpu().numpy() & nat.RM_E_ASYM_NOCONV).any()
    d = (K1 - K0).abs().max().item() / max(1.0, K0.abs().max().item())
    log("uncoupled expansion vs Coulomb matching at A = 400: %.2e" % d)
    assert d < 1e-9
    with pytest.raises(nat.RmError) as ex:
        nat.rm_sweep_energies([h], 8, E, nat.make_opts(solve_fp32=1))
    assert ex.value.code == nat.RM_ERR_ARG
    nat.rm_set_gailitis(h, 0)
    K2, _, _, _ = nat.rm_kmatrix(h, E)
    assert torch.equal(K2, K0)
    h.free()


def test_expansion_beside_a_plain_symmetry_and_in_a_plan(torch_dev, nat):
    """Two symmetries in one sweep, one matched to the expansion at A and
    one matched at a (their workspaces differ in size), against the sum of
    the oracle's two sweeps; then the same sweep captured in a plan and
    replayed twice equals the eager sweep bit for bit."""
    import oracle
    torch, dev = torch_dev
    w = wl.config1()
    sym1 = w.syms[0].as_dict()
    rng = np.random.default_rng(44)
    s2 = wl.random_symmetry(rng, 5, 150, -2.0, 50.0, mesh=w.mesh_spec,
                            thresholds=[0.1, 0.3, 0.5, 0.7, 0.9, 1.1, 1.3, 1.5],
                            target=[0, 2, 2, 4, 6])
    h1 = nat.load_symmetry(w.syms[0])
    h2 = nat.load_symmetry(s2)
    prop = {"A": 120.0, "n_sec": 150, "beta": _beta(8, 5, (0.3, 0.6)),
            "gailitis_terms": 40}
    nat.rm_set_propagation(h1, prop["A"], prop["n_sec"], prop["beta"])
    nat.rm_set_gailitis(h1, prop["gailitis_terms"])
    E = w.mesh[5::37]
    Ed = _dev(torch, dev, E)
    om, st = nat.rm_sweep_energies([h2, h1], 8, Ed, nat.make_opts(chunk=23))
    ref1, _ = outer.sweep_propagated_gailitis(sym1, prop, E, n_target=8)
    ref2 = oracle.sweep(s2.as_dict(), E, n_target=8)["omega"]
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref1 + ref2)
    log("expansion beside a plain symmetry, %d energies: %.2e" % (E.size, err))
    assert err < 1e-6
    plan = nat.Plan([h2, h1], 8, Ed, nat.make_opts(chunk=23))
    for _ in range(2):
        pom, pst = plan.execute()
        torch.cuda.synchronize()
        assert torch.equal(pom, om) and torch.equal(pst, st)
    plan.free()
    h1.free()
    h2.free()


def test_kmatrix_levels_target_converged(torch_dev, nat):
    """The 200-channel, 10-level target of the expansion leg (groups of 20
    degenerate channels with dipole coupling inside them), A = 200 through
    90 sectors, at energies where every column converges (no flags on
    either side).  K here is sensitive (a relative change of 1e-15 in R(a)
    or in the sectors' eigenvalues moves it by 1e-10, measured with the
    oracle), and the two propagations' rounding differs by about 3.5e-10 of
    max(1, |K|) per sector: from the device's own R(a), 2.3e-9 at 10
    sectors, 8.8e-9 at 30 and 3.2e-8 at 90, the same with the expansion
    switched off (so none of it is the expansion's).  Hence: from the
    device's R(a), the oracle's propagation, expansion and matching give K
    within 1e-9 per sector; end to end, within 1e-6."""
    from oracle.rmatrix import channel_data
    torch, dev = torch_dev
    w = wl.outer_levels(M=2048)
    sym = w.syms[0].as_dict()
    h = nat.load_symmetry(w.syms[0])
    prop = {"A": sym["a"] + 180.0, "n_sec": 90,
            "beta": wl.outer_coupling(200), "gailitis_terms": 40}
    nat.rm_set_propagation(h, prop["A"], prop["n_sec"], prop["beta"])
    nat.rm_set_gailitis(h, prop["gailitis_terms"])
    E = w.mesh[[700, 1300, 1900]]  # 6.8, 12.7, 18.6 Ry: all channels open
    K, no, R, st = nat.rm_kmatrix(h, _dev(torch, dev, E), want_R=True)
    K, no, R, st = (K.cpu().numpy(), no.cpu().numpy(), R.cpu().numpy(),
                    st.cpu().numpy())
    secs = outer.outer_sectors(sym, prop)
    A = prop["A"]
    after, end = 0.0, 0.0
    for m, Ee in enumerate(E):
        Kr, P, fl = outer.k_matrix_propagated_gailitis(sym, prop, Ee)
        assert no[m] == P.size == 200
        assert not fl and not (st[m] & nat.RM_E_ASYM_NOCONV)
        RA = outer.propagate(sym["a"] * R[m], secs, Ee) / A
        S, C, Sp, Cp, P2, _ = outer.gailitis(Ee, sym["e_thr"], sym["l"],
                                             sym["z"], prop["beta"], A, 40)
        cd = channel_data(np.array([Ee]), sym["e_thr"], sym["l"], sym["z"], A)
        Kd = outer.k_matrix_asymptotic(RA, A, S, C, Sp, Cp, P2, cd["L"][0])
        Kd = 0.5 * (Kd + Kd.T)
        Kg = K[m, :P.size, :P.size]
        sc = max(1.0, np.abs(Kr).max())
        after = max(after, np.abs(Kg - Kd).max() / sc)
        end = max(end, np.abs(Kg - Kr).max() / sc)
    log("expansion K, 10-level target, converged: %.2e from the device's "
        "R(a), %.2e end to end" % (after, end))
    assert after < 1e-9 * prop["n_sec"]
    assert end < 1e-6
    h.free()


def test_expansion_uncoupled_high_l_and_charge(torch_dev, nat):
    """Channels up to l = 12 with z = 5 (|eta| up to about 4), no
    multipoles, A = 1500: the device's series and Coulomb phase reproduce
    the Coulomb matching at A (its continued fractions) to 1e-9."""
    torch, dev = torch_dev
    rng = np.random.default_rng(31)
    s = wl.random_symmetry(rng, 6, 80, -2.0, 40.0, z=5.0, lmax=12,
                           mesh=(3.0, 10.0, 64))
    h = nat.load_symmetry(s)
    E = _dev(torch, dev, wl.uniform_mesh(3.0, 10.0, 64))
    nat.rm_set_propagation(h, 1500.0, 40)
    K0, _, _, _ = nat.rm_kmatrix(h, E)
    nat.rm_set_gailitis(h, 60)
    K1, _, _, st = nat.rm_kmatrix(h, E)
    assert not (st.cpu().numpy() & nat.RM_E_ASYM_NOCONV).any()
    d = (K1 - K0).abs().max().item() / max(1.0, K0.abs().max().item())
    log("uncoupled expansion, l <= 12, z = 5, A = 1500: %.2e (l %s)"
        % (d, s.l.tolist()))
    assert d < 1e-9
    h.free()


@pytest.mark.parametrize("scales", [(0.3,), (0.3, 0.6, 1.2)])
def test_sweep_with_expansion_other_multipole_orders(torch_dev, nat, scales):
    """Dipole only (lmax = 1) and up to octupole (lmax = 3: a ring of four
    orders, the stacked couplings 3n wide): Omega and flags as the oracle's."""
    torch, dev = torch_dev
    w = wl.config1()
    sym = w.syms[0].as_dict()
    h = nat.load_symmetry(w.syms[0])
    prop = {"A": 120.0, "n_sec": 150, "beta": _beta(8, 9, scales),
            "gailitis_terms": 40}
    nat.rm_set_propagation(h, prop["A"], prop["n_sec"], prop["beta"])
    nat.rm_set_gailitis(h, prop["gailitis_terms"])
    E = w.mesh[3::41]
    om, st = nat.rm_sweep_energies([h], 8, _dev(torch, dev, E),
                                   nat.make_opts(chunk=29))
    ref, flags = outer.sweep_propagated_gailitis(sym, prop, E, n_target=8)
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref)
    got = (st.cpu().numpy() & nat.RM_E_ASYM_NOCONV) != 0
    log("expansion, lmax %d, %d energies: %.2e; flagged %d (oracle %d)"
        % (len(scales), E.size, err, int(got.sum()), int(flags.sum())))
    assert err < 1e-6
    assert np.array_equal(got, flags)
    h.free()


@pytest.mark.parametrize("prec", ["RM_PREC_FP32", "RM_PREC_BF16X3"])
def test_sweep_with_expansion_mixed_pole_sum(torch_dev, nat, prec):
    """The mixed-precision pole sums (FP32 or split-BF16 far poles, FP64
    near ones) under the propagation and the expansion: Omega within the
    mixed path's 1e-4 of the FP64 oracle, flags as the oracle's."""
    torch, dev = torch_dev
    w = wl.config1()
    sym = w.syms[0].as_dict()
    h = nat.load_symmetry(w.syms[0])
    prop = {"A": 120.0, "n_sec": 150, "beta": _beta(8, 1, (0.3, 0.6)),
            "gailitis_terms": 40}
    nat.rm_set_propagation(h, prop["A"], prop["n_sec"], prop["beta"])
    nat.rm_set_gailitis(h, prop["gailitis_terms"])
    E = w.mesh[7::31]
    om, st = nat.rm_sweep_energies([h], 8, _dev(torch, dev, E),
                                   nat.make_opts(prec=getattr(nat, prec),
                                                 near_delta=1e-3))
    ref, flags = outer.sweep_propagated_gailitis(sym, prop, E, n_target=8)
    err, _, _ = omega_normwise_err(om.cpu().numpy(), ref)
    got = (st.cpu().numpy() & nat.RM_E_ASYM_NOCONV) != 0
    log("expansion, %s pole sum, %d energies: %.2e; flagged %d (oracle %d)"
        % (prec, E.size, err, int(got.sum()), int(flags.sum())))
    assert err < 1e-4
    assert np.array_equal(got, flags)
    h.free()
