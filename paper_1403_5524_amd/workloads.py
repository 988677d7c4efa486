"""Seeded synthetic inputs for the outer-region sweep.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic, so both the HIP path and the CPU oracle can be fed from
it.  The paper's own workloads (B II, Ca II, Fe III; Sec. 3 Tables 1-2,
Sec. 6 Table 3) need inner-region data that is not published; these seeded
systems stand in for them with the same kind of shape: n channels, N_H poles
per symmetry (N_H ~ 30-60 n), a fine uniform energy mesh (Sec. 3 asks for
millions of points at meV resolution).

Conventions (units Ry and a0):
* "M energies uniform in [lo, hi]" is the midpoint grid
  E_m = lo + (m + 1/2)(hi - lo)/M.
* poles: i.i.d. uniform draws, sorted ascending; amplitudes w_ik ~ N(0, s^2);
  thresholds ~ U[0, 2]; l ~ U{0..5}; numpy PCG64 with the stated seed, drawn
  in the order poles, amplitudes, thresholds, l.
* a threshold or pole closer than 1e-9 Ry to a mesh point is redrawn, so no
  energy sits on a threshold or on a pole.
"""
from dataclasses import dataclass, field

import numpy as np

MIN_GAP = 1e-9


def uniform_mesh(lo, hi, M):
    """Midpoint grid of M energies on [lo, hi]."""
    return lo + (np.arange(M, dtype=np.float64) + 0.5) * ((hi - lo) / M)


def _mesh_gap(x, lo, hi, M):
    h = (hi - lo) / M
    idx = np.clip(np.rint((x - lo) / h - 0.5), 0, M - 1)
    return np.abs(x - (lo + (idx + 0.5) * h))


def _redraw_near_mesh(x, draw, mesh):
    if mesh is None:
        return x
    lo, hi, M = mesh
    bad = _mesh_gap(x, lo, hi, M) < MIN_GAP
    while bad.any():
        x[bad] = draw(int(bad.sum()))
        bad = _mesh_gap(x, lo, hi, M) < MIN_GAP
    return x


@dataclass
class Symmetry:
    """One LS-pi / J-pi symmetry: what the inner region hands to the sweep."""
    E_pole: np.ndarray          # [N_H] ascending
    w: np.ndarray               # [n, N_H] row-major, w[i, k] = w_ik
    e_thr: np.ndarray           # [n]
    l: np.ndarray               # [n] int32
    a: float = 20.0
    z: float = 1.0
    g: float = 1.0
    target: np.ndarray = None   # [n] int32 or None (identity)

    @property
    def n(self):
        return self.e_thr.size

    @property
    def n_poles(self):
        return self.E_pole.size

    def as_dict(self):
        return {"E_pole": self.E_pole, "w": self.w, "a": self.a,
                "e_thr": self.e_thr, "l": self.l, "z": self.z, "g": self.g,
                "target": self.target}


@dataclass
class Workload:
    name: str
    syms: list
    mesh: np.ndarray
    n_target: int
    mesh_spec: tuple = field(default=None)


def random_symmetry(rng, n, n_poles, pole_lo, pole_hi, w_sigma=0.1, a=20.0,
                    z=1.0, g=1.0, e_lo=0.0, e_hi=2.0, lmax=5, mesh=None,
                    thresholds=None, target=None):
    """Draw one symmetry.  ``thresholds``/``target`` override the per-channel
    threshold draw with shared target levels (batched workloads)."""
    def poles(k):
        return rng.uniform(pole_lo, pole_hi, size=k)
    E_pole = _redraw_near_mesh(poles(n_poles), poles, mesh)
    E_pole.sort()
    w = rng.normal(0.0, w_sigma, size=(n, n_poles))
    if thresholds is None:
        def thr(k):
            return rng.uniform(e_lo, e_hi, size=k)
        e_thr = _redraw_near_mesh(thr(n), thr, mesh)
    else:
        e_thr = np.asarray(thresholds, dtype=np.float64)[target]
    l = rng.integers(0, lmax + 1, size=n).astype(np.int32)
    return Symmetry(E_pole=E_pole, w=np.ascontiguousarray(w), e_thr=e_thr,
                    l=l, a=a, z=z, g=g,
                    target=None if target is None else
                    np.asarray(target, dtype=np.int32))


def single(n, n_poles, pole_lo, pole_hi, mesh_lo, mesh_hi, M, seed,
           name="single", w_sigma=0.1):
    rng = np.random.default_rng(seed)
    spec = (mesh_lo, mesh_hi, M)
    sym = random_symmetry(rng, n, n_poles, pole_lo, pole_hi, w_sigma=w_sigma,
                          mesh=spec)
    return Workload(name, [sym], uniform_mesh(*spec), n, spec)


def config1():
    """8 channels, 200 poles in [-2, 50], 2000 energies in [0, 10], seed 1."""
    return single(8, 200, -2.0, 50.0, 0.0, 10.0, 2000, 1, "c1_n8_nh200_m2000")


def config2(M=100000):
    """200 channels, 8000 poles in [-5, 200], 1e5 energies in [0, 20], seed 2."""
    return single(200, 8000, -5.0, 200.0, 0.0, 20.0, M, 2,
                  "c2_n200_nh8000_m%d" % M)


def config3(M=50000, n_sym=40, n_target=20, seed=3):
    """40 symmetries, n_s log-uniform in [20, 600], N_H = 30 n_s, 20 shared
    target levels with thresholds U[0, 2], one mesh of M energies in [0, 15],
    g_s = 1 + (s mod 10)."""
    rng = np.random.default_rng(seed)
    spec = (0.0, 15.0, M)
    ns = np.rint(np.exp(rng.uniform(np.log(20.0), np.log(600.0),
                                    size=n_sym))).astype(int)

    def thr(k):
        return rng.uniform(0.0, 2.0, size=k)
    levels = np.sort(_redraw_near_mesh(thr(n_target), thr, spec))
    syms = []
    for s, n in enumerate(ns):
        target = rng.integers(0, n_target, size=n)
        syms.append(random_symmetry(rng, int(n), 30 * int(n), -5.0, 200.0,
                                    g=float(1 + s % 10), mesh=spec,
                                    thresholds=levels, target=target))
    return Workload("c3_batched_%dsym_m%d" % (n_sym, M), syms,
                    uniform_mesh(*spec), n_target, spec)


def config4(M=20000):
    """1500 channels, 40000 poles in [-5, 200], 2e4 energies in [0, 20], seed 4."""
    return single(1500, 40000, -5.0, 200.0, 0.0, 20.0, M, 4,
                  "c4_n1500_nh40000_m%d" % M)


def photo_b2(M=409600):
    """Stand-in for the B II K-shell photoionization run (Sec. 3, Table 1:
    400 coupled channels, 409,600 energies): one final symmetry of 400
    channels and 24,800 poles (62 per channel, the ratio of the Sec. 6
    Table 3 shapes) in [-5, 200], thresholds U[0, 2], M energies in [0, 20],
    seed 5; bound-free dipoles d_k ~ N(0, 1) from seed 105; initial state
    at e0 = -0.8 Ry.  Returns (workload, dipoles, e0)."""
    w = single(400, 24800, -5.0, 200.0, 0.0, 20.0, M, 5,
               "b2_photo_n400_nh24800_m%d" % M)
    dip = np.random.default_rng(105).normal(size=24800)
    return w, dip, -0.8


def radiative_widths(n_poles, seed, lo=1e-6, hi=1e-3):
    """Radiative widths Gamma_k of the inner-region states for the damped
    photoionization: log-uniform in [lo, hi] Ry (inner-shell radiative
    widths run from micro- to milli-Rydberg), numpy PCG64 with the seed."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=n_poles)


def photo_ca2(M=6000):
    """Stand-in for the Ca II photoionization run (Sec. 3, Table 2: 513
    target states, 1815 coupled channels, Hamiltonian dimension 23,073,
    6,000 energies): one final symmetry of 1815 channels and 23,073 poles
    in [-5, 200], thresholds U[0, 2], M energies in [0, 20], seed 7;
    bound-free dipoles d_k ~ N(0, 1) from seed 107; initial state at
    e0 = -0.8 Ry.  Returns (workload, dipoles, e0)."""
    w = single(1815, 23073, -5.0, 200.0, 0.0, 20.0, M, 7,
               "ca2_photo_n1815_nh23073_m%d" % M)
    dip = np.random.default_rng(107).normal(size=23073)
    return w, dip, -0.8


# The ten (channels n, poles m) shapes of the paper's Sec. 6 Table 3 (the
# R-matrix formation of PSTGF for e- + Fe III), m/n ~ 62 throughout.
TABLE3_SHAPES = [(267, 16512), (308, 19201), (399, 24666), (526, 32530),
                 (132, 8155), (260, 16102), (837, 51573), (796, 49169),
                 (1368, 84321), (1241, 76646)]


def table3_symmetry(n, m, M, seed=8):
    """One symmetry of a Table 3 shape with the c2 distributions (poles
    U[-5, 200], w ~ N(0, 0.1^2), thresholds U[0, 2], l ~ U{0..5}) and the
    M-point mesh on [0, 20] it is evaluated on; seed + n."""
    rng = np.random.default_rng(seed + n)
    sym = random_symmetry(rng, n, m, -5.0, 200.0, mesh=(0.0, 20.0, M))
    return sym, uniform_mesh(0.0, 20.0, M)


def outer_levels(n=200, n_levels=10, spacing=0.5, n_poles=8000, M=2048,
                 seed=9):
    """200 channels on 10 target levels spaced 0.5 Ry (20 channels of
    random l per level, channel c on level c mod 10), 8000 poles in
    [-5, 200], M energies in [0, 20]: a target whose levels lie far enough
    apart for the asymptotic expansion beyond A, seeded."""
    rng = np.random.default_rng(seed)
    spec = (0.0, 20.0, M)
    levels = spacing * np.arange(n_levels)
    target = np.arange(n) % n_levels
    sym = random_symmetry(rng, n, n_poles, -5.0, 200.0, mesh=spec,
                          thresholds=levels, target=target)
    return Workload("levels_n%d_t%d_nh%d_m%d" % (n, n_levels, n_poles, M),
                    [sym], uniform_mesh(*spec), n_levels, spec)


def outer_coupling(n, lmax=2, seed=6, scales=(1.0, 4.0)):
    """Long-range multipole coefficients beta [lmax, n, n] (symmetric,
    N(0, scale^2) off and on the diagonal; lam = 1 dipole, 2 quadrupole) for
    the outer-region propagation, seeded."""
    rng = np.random.default_rng(seed)
    out = []
    for lam in range(lmax):
        M = rng.normal(0.0, scales[lam], (n, n))
        out.append(0.5 * (M + M.T))
    return np.stack(out)


def inner_model(n=8, seed=21, a=20.0, z=1.0, lmax=3):
    """Model inner region of n channels on [0, a]: thresholds ~ U[0, 2]
    sorted (the first at 0), l ~ U{0..lmax}, a symmetric Gaussian coupling
    matrix with diagonal depths ~ U[1, 4] Ry, off-diagonal ~ U[0.1, 1] Ry,
    ranges ~ U[1.5, 4] a0 (symmetrised), drawn in that order from PCG64."""
    rng = np.random.default_rng(seed)
    e = np.sort(rng.uniform(0.0, 2.0, n))
    e[0] = 0.0
    l = rng.integers(0, lmax + 1, n)
    off = rng.uniform(0.1, 1.0, (n, n))
    depth = 0.5 * (off + off.T)
    depth[np.arange(n), np.arange(n)] = rng.uniform(1.0, 4.0, n)
    rg = rng.uniform(1.5, 4.0, (n, n))
    return {"e_thr": e, "l": l, "z": float(z), "a": float(a),
            "depth": depth, "range": 0.5 * (rg + rg.T)}


def tiny(n=3, n_poles=12, M=40, seed=11, pole_lo=-2.0, pole_hi=30.0,
         mesh_lo=0.0, mesh_hi=6.0):
    """Small system for quick checks."""
    return single(n, n_poles, pole_lo, pole_hi, mesh_lo, mesh_hi, M, seed,
                  "tiny_n%d_nh%d_m%d" % (n, n_poles, M))


def sample_indices(M, count, seed=0):
    """Seeded sorted subset of mesh indices (for oracle comparisons)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(M, size=min(count, M), replace=False))


def narrow_resonance_system(seed, n=200, n_poles=8000, n_narrow=50,
                            pole_lo=-5.0, pole_hi=200.0, mesh_lo=0.0,
                            mesh_hi=20.0, M_fine=1000000, width_lo=1e-5,
                            width_hi=1e-3):
    """C2-style symmetry plus n_narrow injected weakly coupled poles.

    Each injected pole sits uniformly in the open part of [mesh_lo, mesh_hi]
    with amplitude vector c u (u a random unit vector).  c^2 is drawn so that
    a crude width proxy c^2 * mean_i sqrt(E_r - e_i)_+ lands log-uniformly in
    [width_lo, width_hi]; the nominal (E_r, proxy width) pairs are returned
    as the truth list.  Poles and thresholds avoid the fine mesh by 1e-9.
    """
    rng = np.random.default_rng(seed)
    spec = (mesh_lo, mesh_hi, M_fine)
    base = random_symmetry(rng, n, n_poles, pole_lo, pole_hi, mesh=spec)

    def pos(k):
        return rng.uniform(max(mesh_lo, 2.2), mesh_hi - 0.1, size=k)
    Er = _redraw_near_mesh(pos(n_narrow), pos, spec)
    widths = np.exp(rng.uniform(np.log(width_lo), np.log(width_hi),
                                size=n_narrow))
    u = rng.normal(size=(n, n_narrow))
    u /= np.linalg.norm(u, axis=0, keepdims=True)
    kbar = np.sqrt(np.clip(Er[None, :] - base.e_thr[:, None], 0.0, None))
    proxy = (kbar * u * u).sum(axis=0)
    c = np.sqrt(widths / np.maximum(proxy, 1e-12))
    E_all = np.concatenate([base.E_pole, Er])
    w_all = np.concatenate([base.w, u * c[None, :]], axis=1)
    order = np.argsort(E_all, kind="stable")
    E_all = E_all[order]
    w_all = np.ascontiguousarray(w_all[:, order])
    # keep poles strictly ascending
    if np.any(np.diff(E_all) <= 0):
        raise ValueError("coincident poles; change the seed")
    sym = Symmetry(E_pole=E_all, w=w_all, e_thr=base.e_thr, l=base.l,
                   a=base.a, z=base.z, g=base.g)
    truth = np.stack([Er, widths], axis=1)
    return sym, truth, spec
