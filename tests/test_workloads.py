"""Seeded generators: determinism, shapes and the no-pole/no-threshold-on-mesh rule."""
import numpy as np

from paper_1403_5524_amd import workloads as wl


def test_config1_deterministic_and_shaped():
    a, b = wl.config1(), wl.config1()
    sa, sb = a.syms[0], b.syms[0]
    assert sa.w.shape == (8, 200) and sa.E_pole.shape == (200,)
    assert np.array_equal(sa.w, sb.w) and np.array_equal(sa.E_pole, sb.E_pole)
    assert np.all(np.diff(sa.E_pole) > 0)
    assert a.mesh.size == 2000 and abs(a.mesh[0] - 0.0025) < 1e-15


def test_no_pole_or_threshold_on_mesh():
    w = wl.config1()
    s = w.syms[0]
    gap_p = np.abs(w.mesh[:, None] - s.E_pole[None, :]).min()
    gap_t = np.abs(w.mesh[:, None] - s.e_thr[None, :]).min()
    assert gap_p >= wl.MIN_GAP and gap_t >= wl.MIN_GAP


def test_config3_shapes():
    w = wl.config3(M=100)
    assert len(w.syms) == 40 and w.n_target == 20
    ns = np.array([s.n for s in w.syms])
    assert ns.min() >= 20 and ns.max() <= 600
    for s in w.syms:
        assert s.n_poles == 30 * s.n and s.target.max() < 20
    assert sorted({s.g for s in w.syms}) == [float(v) for v in range(1, 11)]
