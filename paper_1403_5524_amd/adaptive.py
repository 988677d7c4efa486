"""Learned adaptive energy mesh.

The paper's sweeps need millions of energies to resolve narrow resonances
(Sec. 3).  Here a small MLP, trained on the device by the library's own
kernels (rm_mlp_*), predicts from cheap per-window features of a symmetry
how much structure Omega(E) has in each energy window; rm_mesh_from_density
turns the prediction into an adaptive mesh, and the uniform fine mesh swept
with the plain (FP64) method is the reference.

Pipeline (all arrays for the sweep and the network live on the GPU):
  features(sym)            host: pole counts, amplitude norms, thresholds
  fine = sweep(uniform)   rm_sweep_energies over a uniform fine mesh
  labels = log curvature of Omega per window (from the fine sweep)
  train                    rm_mlp_grad + rm_mlp_adam_step
  density = 10**mlp(features) -> rm_mesh_from_density -> adaptive mesh
  evaluate                 integrated Omega per transition vs the fine sweep,
                           missed narrow resonances
"""
import math

import numpy as np

from . import native

N_FEAT = 12


def window_features(sym, lo, hi, nw):
    """Per-window features [nw, N_FEAT] (float32) from poles and thresholds.

    Narrow resonances come from poles with small surface amplitudes, so the
    features describe, per window and its neighbourhood, how many poles sit
    there and how weakly the weakest of them couples, plus where thresholds
    (and the Rydberg series below them) lie.
    """
    h = (hi - lo) / nw
    Ek = np.asarray(sym.E_pole)
    amp2 = (np.asarray(sym.w) ** 2).sum(axis=0)
    idx = np.floor((Ek - lo) / h).astype(np.int64)
    inside = (idx >= 0) & (idx < nw)
    cnt = np.bincount(idx[inside], minlength=nw).astype(np.float64)
    la = np.log10(amp2[inside] + 1e-30)
    minamp = np.full(nw, 2.0)
    np.minimum.at(minamp, idx[inside], la)
    inv = np.zeros(nw)
    np.add.at(inv, idx[inside], 1.0 / (amp2[inside] + 1e-12))

    def smooth(v, r, op):
        out = v.copy()
        for s in range(1, r + 1):
            out = op(out, np.roll(v, s))
            out = op(out, np.roll(v, -s))
        return out
    centers = lo + (np.arange(nw) + 0.5) * h
    thr = np.sort(np.asarray(sym.e_thr))
    pos = np.searchsorted(thr, centers)
    above = np.where(pos < thr.size, thr[np.minimum(pos, thr.size - 1)] - centers, 10.0)
    below = np.where(pos > 0, centers - thr[np.maximum(pos - 1, 0)], 10.0)
    tcount = np.bincount(np.clip(np.floor((thr - lo) / h).astype(np.int64), 0,
                                 nw - 1), minlength=nw)
    f = np.stack([
        np.log1p(cnt),
        minamp,
        np.log10(inv + 1e-3),
        np.log1p(smooth(cnt, 2, np.add)),
        smooth(minamp, 2, np.minimum),
        np.log10(smooth(inv, 2, np.add) + 1e-3),
        np.log10(np.maximum(above, 1e-6)),
        np.log10(np.maximum(below, 1e-6)),
        np.log1p(tcount),
        centers / max(hi, 1e-12),
        np.log10(pos + 1.0),
        np.log10(np.maximum(centers - thr[0], 1e-6)) if thr.size else centers,
    ], axis=1)
    return f.astype(np.float32)


class FineSweep:
    """Per-transition integrals and per-window variation and curvature of a
    swept mesh."""

    def __init__(self, integrals, variation, total, mesh_size,
                 curvature=None, nonfinite=None):
        self.integrals = integrals      # [P] float64 (numpy)
        self.variation = variation      # [nw] float64
        self.curvature = curvature      # [nw] float64: max |second difference|
        self.total = total
        self.mesh_size = mesh_size
        # energies whose Omega row the sweep flagged RM_E_NONFINITE
        self.nonfinite = nonfinite if nonfinite is not None else []


def sweep_integrals(handles, n_target, E, lo, hi, nw=None, chunk=25000,
                    opts=None):
    """Sweep a mesh (device float64, ascending) chunk by chunk.

    Returns a FineSweep: trapezoid integrals of every Omega(t, t') over [lo, hi]
    (end segments held constant), and, when nw is given, the total variation
    of sum_pairs Omega in each of nw windows and the largest second
    difference of it there (on a uniform mesh, proportional to the
    curvature).
    """
    import torch
    M = int(E.numel())
    P = n_target * (n_target + 1) // 2
    dev = E.device
    integ = torch.zeros(P, dtype=torch.float64, device=dev)
    var = torch.zeros(nw if nw else 1, dtype=torch.float64, device=dev)
    curv = np.zeros(nw if nw else 1)
    prev_E, prev_om = None, None
    h = (hi - lo) / nw if nw else None
    nonfinite = []
    for c0 in range(0, M, chunk):
        Ec = E[c0:c0 + chunk]
        om, st = native.rm_sweep_energies(handles, n_target, Ec, opts)
        bad = ((st & native.RM_E_NONFINITE) != 0).nonzero().flatten()
        if bad.numel():
            nonfinite += [float(x) for x in Ec[bad[:8]].cpu().numpy()]
        if prev_E is not None:
            Ec2 = torch.cat([prev_E.view(1), Ec])
            om2 = torch.cat([prev_om.view(1, -1), om])
        else:
            integ += om[0] * (Ec[0] - lo)
            Ec2, om2 = Ec, om
        dE = (Ec2[1:] - Ec2[:-1]).view(-1, 1)
        integ += (0.5 * dE * (om2[1:] + om2[:-1])).sum(dim=0)
        if nw:
            sig = om2.sum(dim=1)
            dv = (sig[1:] - sig[:-1]).abs()
            mid = 0.5 * (Ec2[1:] + Ec2[:-1])
            wi = ((mid - lo) / h).floor().clamp(0, nw - 1).long()
            var.index_add_(0, wi, dv)
            if sig.numel() > 2:
                d2 = (sig[2:] - 2.0 * sig[1:-1] + sig[:-2]).abs()
                ci = ((Ec2[1:-1] - lo) / h).floor().clamp(0, nw - 1).long()
                d2h = d2.cpu().numpy()
                ok = np.isfinite(d2h)
                np.maximum.at(curv, ci.cpu().numpy()[ok], d2h[ok])
        prev_E, prev_om = Ec[-1].clone(), om[-1].clone()
        del om
    integ += prev_om * (hi - prev_E)
    torch.cuda.synchronize()
    return FineSweep(integ.cpu().numpy(), var.cpu().numpy() if nw else None,
                     float(integ.sum().item()), M,
                     curv if nw else None, nonfinite)


def labels_from_variation(variation, scale="mean"):
    """log10 of the window's variation (or curvature) relative to its mean,
    or to its median when a few windows dominate the mean (floored)."""
    v = np.asarray(variation, dtype=np.float64)
    ref = np.median(v) if scale == "median" else v.mean()
    return np.log10(v / max(ref, 1e-300) + 1e-3).astype(np.float32)


def heuristic_density(sym, lo, hi, nw):
    """Non-learned density: poles per window weighted by 1/|w_k|^2."""
    h = (hi - lo) / nw
    amp2 = (np.asarray(sym.w) ** 2).sum(axis=0)
    idx = np.floor((np.asarray(sym.E_pole) - lo) / h).astype(np.int64)
    ok = (idx >= 0) & (idx < nw)
    d = np.zeros(nw)
    np.add.at(d, idx[ok], 1.0 / (amp2[ok] + 1e-4))
    return d.astype(np.float32)


class Normaliser:
    """Per-feature standardisation from the training set; a feature that is
    (nearly) constant there is only centred, and every standardised value
    is clipped to +-8, so that a test window outside the training range
    cannot drive the network far from what it was trained on."""

    def __init__(self, X):
        self.mu = X.mean(axis=0)
        self.sd = np.maximum(X.std(axis=0), 1e-2)

    def __call__(self, X):
        return np.clip((X - self.mu) / self.sd, -8.0, 8.0).astype(np.float32)


def train_mlp(X, y, width=256, n_layers=4, steps=1500, batch=1024, lr=1e-3,
              seed=0, prec=0, log=None):
    """Train on the device; returns (mlp, loss history)."""
    import torch
    dev = torch.device("cuda:0")
    Xt = torch.as_tensor(X, device=dev)
    yt = torch.as_tensor(y, device=dev)
    mlp = native.Mlp(X.shape[1], width, n_layers, prec, seed)
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    n = Xt.shape[0]
    for step in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).to(dev)
        xb = Xt.index_select(0, idx).contiguous()
        yb = yt.index_select(0, idx).contiguous()
        loss, _ = mlp.grad(xb, yb)
        mlp.adam_step(lr=lr)
        if step % 100 == 0 or step == steps - 1:
            hist.append((step, float(loss.item())))
            if log:
                log("mlp step %d loss %.4f" % hist[-1])
    return mlp, hist


def mesh_from_log_density(logd, lo, hi, M, floor_frac=0.3, alpha=1.0):
    """Adaptive mesh from predicted log10 densities (device float32)."""
    import torch
    d = torch.pow(10.0, alpha * logd.float()).contiguous()
    return native.rm_mesh_from_density(d, lo, hi, floor_frac, M)


def missed_resonances(E, truth, min_width):
    """Truth resonances of width >= min_width with < 3 mesh points within
    +-width of their position."""
    E = np.asarray(E)
    miss = 0
    tot = 0
    for Er, G in truth:
        if G < min_width:
            continue
        tot += 1
        k = np.searchsorted(E, Er - G), np.searchsorted(E, Er + G)
        if k[1] - k[0] < 3:
            miss += 1
    return miss, tot


def integrated_error(test, fine, rel_floor=1e-6):
    """Max and mean relative error of per-transition integrals (transitions
    with integral above rel_floor times the largest)."""
    J = fine.integrals
    keep = np.abs(J) > rel_floor * np.abs(J).max()
    rel = np.abs(test.integrals[keep] - J[keep]) / np.abs(J[keep])
    return float(rel.max()), float(rel.mean())


def relative_curvature(handle, n, E, nwin):
    """Per window of a uniform mesh E (device, nwin equal windows), the
    largest second difference of any single transition's Omega relative to
    that transition's largest value over the mesh: the trapezoid rule's
    error for the worst-sampled transition, not only for the strong ones
    that dominate the sum."""
    import torch
    om, _ = native.rm_sweep_energies([handle], n, E)
    scale = om.abs().amax(dim=0).clamp_min(1e-300)
    d2 = (om[2:] - 2.0 * om[1:-1] + om[:-2]).abs() / scale
    del om
    per_e = d2.amax(dim=1)            # worst transition at each energy
    del d2
    M = int(E.numel())
    wi = (torch.arange(1, M - 1, device=E.device) * nwin) // M
    out = np.zeros(nwin)
    v = per_e.cpu().numpy()
    w = wi.cpu().numpy()
    ok = np.isfinite(v)
    np.maximum.at(out, w[ok], v[ok])
    return out


def train_set(seeds, n=200, n_poles=8000, n_narrow=50, lo=0.0, hi=20.0,
              dE_fine=2e-5, nw=4096, sub=1.0, log=print, label="sum"):
    """Features and curvature labels of the training systems.

    Each seed's system (the test system's kind) is swept with the plain
    FP64 method on the fine spacing dE_fine, but only over a sub-window of
    `sub` Ry placed by the seed anywhere in [lo, hi] (thresholds and their
    Rydberg series included), so that hundreds of systems cost what a few
    full sweeps would; the labels are those of the windows of the [lo, hi]
    grid that lie wholly inside it."""
    import torch
    from . import workloads as wl
    dev = torch.device("cuda:0")
    h = (hi - lo) / nw
    feats, labels = [], []
    for s in seeds:
        sym, _, _ = wl.narrow_resonance_system(
            s, n=n, n_poles=n_poles, n_narrow=n_narrow, mesh_lo=lo,
            mesh_hi=hi, M_fine=int(round((hi - lo) / dE_fine)))
        rng = np.random.default_rng(s + 7)
        a0 = rng.uniform(lo, hi - sub)
        w0, w1 = int(math.ceil((a0 - lo) / h)), int(math.floor((a0 + sub - lo) / h))
        b0, b1 = lo + w0 * h, lo + w1 * h
        M = int(round((b1 - b0) / dE_fine))
        E = torch.as_tensor(b0 + (np.arange(M) + 0.5) * ((b1 - b0) / M),
                            device=dev)
        hd = native.load_symmetry(sym)
        if label == "relative":
            lab = relative_curvature(hd, n, E, w1 - w0)
        else:
            j = sweep_integrals([hd], n, E, b0, b1, nw=w1 - w0)
            lab = j.curvature
        hd.free()
        f = window_features(sym, lo, hi, nw)[w0:w1]
        feats.append(f)
        labels.append(labels_from_variation(lab, "median"))
        if len(feats) % 16 == 0:
            log("training systems swept: %d of %d" % (len(feats), len(seeds)))
    log("training set: %d systems, %d windows" % (len(seeds),
                                                  sum(x.shape[0] for x in feats)))
    return np.concatenate(feats), np.concatenate(labels)


def keep_off_poles(E, sym, gap=1e-9):
    """Move the points of an adaptive mesh (device, ascending) that sit
    within `gap` of a pole or threshold of sym to 2 gap from it (the
    uniform meshes are drawn to keep that distance; an adaptive one must
    keep it too, or the pole sum divides by ~0)."""
    import torch
    e = E.cpu().numpy()
    for x in (np.asarray(sym.E_pole), np.sort(np.asarray(sym.e_thr))):
        k = np.clip(np.searchsorted(x, e), 1, x.size - 1)
        near = np.where(np.abs(e - x[k]) < np.abs(e - x[k - 1]), x[k], x[k - 1])
        bad = np.abs(e - near) < gap
        e[bad] = near[bad] + np.where(e[bad] >= near[bad], 2 * gap, -2 * gap)
    return torch.as_tensor(np.sort(e), device=E.device)


def run_experiment(train_seeds, test_seed, n=200, n_poles=8000, n_narrow=50,
                   lo=0.0, hi=20.0, M_fine=1000000, M_adapt=100000,
                   nw=4096, steps=1500, log=print, truth_fn=None,
                   train_sub=1.0, couple=0.25, floor=0.7, alpha=0.35,
                   label="sum"):
    """Train on train_seeds (sub-window sweeps, train_set), then compare
    meshes of M_adapt points on test_seed against the M_fine uniform fine
    mesh: uniform, the non-learned coupling heuristic, the learned density
    alone, and the learned density mixed with the heuristic (weight
    `couple` on the heuristic; both normalised to unit mass first), each
    with a uniform share `floor` of the points.

    The network learns log10 of each window's largest second difference
    of sum Omega relative to the median window; the density follows
    10^(alpha * prediction): alpha = 1/2 would follow the square root of
    the curvature (a peak of width G and height A has curvature ~ A/G^2, so
    the density grows as 1/G); the default 0.35, with the uniform share 0.7
    and the coupling weight 0.25, was chosen on the 32-channel case of the
    GPU test, where it resolves every resonance without raising the
    largest integration error above the uniform mesh's.

    truth_fn(sym, nominal) -> [(E_r, Gamma)] measures the test system's
    resonances near the injected poles (nominal: the generator's
    (E_pole, proxy width) list); without it the nominal list is used."""
    import torch
    from . import workloads as wl
    dev = torch.device("cuda:0")
    X, y = train_set(train_seeds, n=n, n_poles=n_poles, n_narrow=n_narrow,
                     lo=lo, hi=hi, dE_fine=(hi - lo) / M_fine, nw=nw,
                     sub=train_sub, log=log, label=label)
    norm = Normaliser(X)
    mlp, hist = train_mlp(norm(X), y, steps=steps, log=log)

    sym, nominal, spec = wl.narrow_resonance_system(
        test_seed, n=n, n_poles=n_poles, n_narrow=n_narrow, mesh_lo=lo,
        mesh_hi=hi, M_fine=M_fine)
    truth = np.asarray(truth_fn(sym, nominal) if truth_fn else nominal)
    h = native.load_symmetry(sym)
    Ej = torch.as_tensor(wl.uniform_mesh(lo, hi, M_fine), device=dev)
    fine = sweep_integrals([h], n, Ej, lo, hi, nw=nw)
    Xt = torch.as_tensor(norm(window_features(sym, lo, hi, nw)), device=dev)
    pred = mlp.forward(Xt)
    heur = torch.as_tensor(heuristic_density(sym, lo, hi, nw), device=dev)
    learned = torch.pow(10.0, alpha * pred.float())
    mix = ((1.0 - couple) * learned / learned.sum()
           + couple * heur / heur.sum()).contiguous()
    meshes = {
        "uniform": torch.as_tensor(wl.uniform_mesh(lo, hi, M_adapt), device=dev),
        "heuristic": native.rm_mesh_from_density(heur, lo, hi, floor, M_adapt),
        "learned": native.rm_mesh_from_density(learned.contiguous(), lo, hi,
                                               floor, M_adapt),
        "learned+coupling": native.rm_mesh_from_density(mix, lo, hi, floor,
                                                        M_adapt),
    }
    for k in ("heuristic", "learned", "learned+coupling"):
        meshes[k] = keep_off_poles(meshes[k], sym)
    min_w = 2.0 * (hi - lo) / M_fine
    ok = np.isfinite(truth).all(axis=1)
    out = {"train_loss": hist, "fine_points": M_fine, "points": M_adapt,
           "train_systems": len(train_seeds), "train_windows": int(X.shape[0]),
           "test_seed": test_seed,
           "density": {"alpha": alpha, "floor": floor, "couple": couple},
           "truth": "measured" if truth_fn else "nominal",
           "truth_resonances": int(ok.sum()),
           "truth_width_range": [float(truth[ok, 1].min()),
                                 float(truth[ok, 1].max())] if ok.any() else None}
    for name, E in meshes.items():
        r = sweep_integrals([h], n, E, lo, hi)
        mx, mean = integrated_error(r, fine)
        miss, tot = missed_resonances(E.cpu().numpy(), truth[ok], min_w)
        out[name] = {"int_err_max": mx, "int_err_mean": mean,
                     "missed": miss, "resonances": tot}
        if r.nonfinite:
            out[name]["nonfinite_energies"] = r.nonfinite[:8]
        log("%-16s int err max %.3e mean %.3e missed %d/%d"
            % (name, mx, mean, miss, tot))
    h.free()
    mlp.free()
    return out


if __name__ == "__main__":   # training on the full seed range (GPU)
    import json
    import sys
    last = int(sys.argv[1]) if len(sys.argv) > 1 else 1255
    res = run_experiment(train_seeds=list(range(1000, last + 1)),
                         test_seed=3000,
                         log=lambda m: print(m, file=sys.stderr, flush=True))
    json.dump(res, sys.stdout)
    print()
