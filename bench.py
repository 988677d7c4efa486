"""Benchmark: energy points per second of the outer-region sweep (K -> Omega)
on the 200-channel, 8000-pole symmetry over a 1e5-point mesh in [0, 20] Ry,
plus the max relative error of Omega against the FP64 CPU oracle.

One step = one rm_sweep_energies call over the whole mesh (channel functions,
pole sum, matching, K, T, Omega for every energy), inputs resident in HBM.
The headline is the plain FP64 path (--prec); the mixed precisions named by
--also are timed on the same workload and reported with their speedup.
Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--prec fp64|fp32|bf16x3]
                    [--also bf16x3,fp32] [--graph] [--workload c2|c3|c4]
                    [--no-postproc] [--photo-M N] [--photo-ca-M N]
                    [--outer-M N] [--inner-N N] [--table3]

After the headline sweep, the sweep's FP64 Omega is smoothed, averaged into
effective collision strengths and summed over level groups; those kernels'
times and rooflines are reported under "postproc".  A photoionization leg
times rm_photoionization on the B II shape of the paper's Table 1 (400
channels, every 50th energy of 409,600) under "photoionization" and on the
Ca II shape of its Table 2 (1815 channels, every 3rd energy of 6000) under
"photoionization_ca2", and an
outer-region leg sweeps the headline symmetry with the R-matrix propagated
through multipole coupling (rm_set_propagation) under "outer_propagation",
and a 200-channel, 10-level target propagated to A = 200 and matched there
to the asymptotic expansion (rm_set_gailitis) under "outer_expansion".
An inner-region leg times the full eigen-solve that supplies poles and
amplitudes (rm_inner_region, 8 channels x 512 sine functions, D = 4096) under
"inner_region", with the oracle's solve of the same model as its CPU baseline.
A learned-mesh leg trains the network on narrow-resonance systems and judges
its 1e5-point adaptive mesh against a 1e6-point uniform sweep under
"learned_mesh".
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}   # TFLOP/s dense MFMA
PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2}

# HBM bytes per energy from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE) of the 200-channel workload, scaled by what the same counters
# read for a plain 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0).
# A figure applies only while its kernel source is the one measured.
PMC_TRAFFIC = {
    "match_kernel": {"src": "paper_1403_5524_amd/csrc/match.hip",
                     "sha256_16": "87d60d344558c9f6",
                     "bytes_per_energy": 23.20e6 + 7.640e6},
    "polesum_fp64": {"src": "paper_1403_5524_amd/csrc/polesum.hip",
                     "sha256_16": "63e41f950c81571c",
                     "bytes_per_energy": 0.1942e6 + 0.3228e6},
    "polesum_bf16x3": {"src": "paper_1403_5524_amd/csrc/polesum_pd.hip",
                       "sha256_16": "045eb073247d461b",
                       "bytes_per_energy": 0.2359e6 + 0.7140e6},
    "polesum_fp32": {"src": "paper_1403_5524_amd/csrc/polesum_pd.hip",
                     "sha256_16": "045eb073247d461b",
                     "bytes_per_energy": 0.2357e6 + 0.7133e6},
}


def measured_traffic(key, energies):
    """HBM bytes for `energies` energies, or None if the kernel changed."""
    import hashlib
    t = PMC_TRAFFIC.get(key)
    if t is None:
        return None
    with open(os.path.join(ROOT, t["src"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha256_16"]:
            return None
    return t["bytes_per_energy"] * energies


def match_flops(n, n_open):
    """Algorithmic FP64 flops of matching one symmetry at energies with
    n_open = m open channels, counted as the minimal dense step: a
    symmetric factorisation of the n x n matrix (n^3/3), forward and back
    substitution of m right-hand sides (2 n^2 m), and the T step on the
    m x m K-matrix (16 m^3 / 3: 1 + K^2, its Cholesky, Z = L^-1 K,
    Y = L^-T Z, Q = Z^T Z)."""
    no = n_open.astype(np.float64)
    f = n ** 3 / 3.0 + 2.0 * n * n * no + (16.0 / 3.0) * no ** 3
    return float(np.where(no > 0, f, 0.0).sum())


def match_flops_executed(n, n_open):
    """The flops the kernel runs at most energies: the LU (2 n^3 / 3 instead
    of n^3/3), the substitutions (2 n^2 m) and its T step (3 m^3: lower
    triangle of 1 + K^2 m^3, Cholesky m^3/3, L^-1 m^3/3, A = L^-T L^-1
    m^3/3, lower triangle of Y = K A m^3; energies with large K take a
    route of 13 m^3 / 3)."""
    no = n_open.astype(np.float64)
    f = (2.0 / 3.0) * n ** 3 + 2.0 * n * n * no + 3.0 * no ** 3
    return float(np.where(no > 0, f, 0.0).sum())


def omega_errors(got, ref):
    """Max relative error of Omega over the sampled energies, two ways:
    normwise per energy (max |dOmega| / max |Omega_ref| of the energy's
    row) and elementwise (|dOmega| / |Omega_ref| over every transition with
    |Omega_ref| at least 1e-8 of its row's largest value)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    row = np.maximum(np.abs(ref).max(axis=1), 1e-300)
    diff = np.abs(got - ref)
    normwise = float((diff.max(axis=1) / row).max())
    big = np.abs(ref) >= 1e-8 * row[:, None]
    rel = np.where(big, diff / np.maximum(np.abs(ref), 1e-300), 0.0)
    return normwise, float(rel.max())


def note(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        info = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        if info:
            return int(info[0]["num_threads"])
    except Exception:
        pass
    return os.cpu_count()


def cpu_baseline_1thread(sym, mesh, count):
    """The same oracle sweep with the BLAS pool held to one thread."""
    import oracle
    from threadpoolctl import threadpool_limits
    idx = np.linspace(0, mesh.size - 1, count).round().astype(int)
    with threadpool_limits(limits=1, user_api="blas"):
        t0 = time.perf_counter()
        oracle.sweep(sym.as_dict(), mesh[idx])
        dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "energies/s", "cores": 1,
            "kind": "oracle", "sample": "%d of %d mesh energies, evenly "
                                        "spaced (%.1f s)" % (count, mesh.size, dt)}


def library_gemm_ceiling(torch, sym, mesh, batch=32, reps=5):
    """Context, not the path: the pole-sum shape (W diag(d)) W^T as a plain
    FP64 library GEMM (torch.matmul, rocBLAS / hipBLASLt) over `batch`
    energies, with W diag(d) formed beforehand; full-square flops."""
    dev = torch.device("cuda:0")
    W = torch.as_tensor(sym.w, dtype=torch.float64, device=dev)      # [n, N_H]
    Wt = W.t().contiguous()                                           # [N_H, n]
    Ek = torch.as_tensor(sym.E_pole, dtype=torch.float64, device=dev)
    Es = torch.as_tensor(mesh[:: max(1, mesh.size // batch)][:batch],
                         dtype=torch.float64, device=dev)
    A = (W[None, :, :] / (Ek[None, None, :] - Es[:, None, None])).contiguous()
    R = torch.matmul(A, Wt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        R = torch.matmul(A, Wt)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    n, nh = sym.w.shape
    flops = 2.0 * n * n * nh * Es.numel()
    del A, R
    return {"kind": "torch.matmul FP64 (rocBLAS / hipBLASLt), context",
            "energies": int(Es.numel()), "ms": dt * 1e3,
            "tflops_full_square": flops / dt / 1e12,
            "energies_per_s_gemm_only": Es.numel() / dt}


def cpu_baseline(sym, mesh, count):
    """The oracle as it stands, timed on this host on a bounded sample.
    Returns the record, the sampled mesh indices and the oracle's Omega
    there (the reference of the error sample)."""
    import oracle
    idx = np.linspace(0, mesh.size - 1, count).round().astype(int)
    t0 = time.perf_counter()
    r = oracle.sweep(sym.as_dict(), mesh[idx])
    dt = time.perf_counter() - t0
    return ({"value": count / dt, "unit": "energies/s",
             "cores": blas_threads(), "kind": "oracle",
             "sample": "%d of %d mesh energies, evenly spaced (%.1f s)"
                       % (count, mesh.size, dt)}, idx, r["omega"])


RYD_EV = 13.605693122994


def postproc_leg(native, torch, E, omega, mesh, e_level, n_t, steps):
    """Time the post-processing of the sweep's Omega: Gaussian smoothing at
    100 meV FWHM, effective collision strengths at 8 temperatures, sums over
    20 groups of levels.  Kernel times come from rm_profile's events."""
    M, P = int(omega.shape[0]), int(omega.shape[1])
    fwhm = 0.1 / RYD_EV
    s = fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))
    lo = np.searchsorted(mesh, mesh - 8.0 * s, side="left")
    hi = np.searchsorted(mesh, mesh + 8.0 * s, side="right")
    conv_flops = 2.0 * float((hi - lo).sum()) * P
    kT = np.geomspace(0.05, 5.0, 8)
    n_g = max(1, n_t // 10)
    group = np.minimum(np.arange(n_t) // 10, n_g - 1)
    Pg = n_g * (n_g + 1) // 2
    out = torch.empty_like(omega)
    calls = {
        "convolve": (lambda: native.rm_convolve_gaussian(E, omega, fwhm, out),
                     "mfma", conv_flops, 78.6, "TFLOP/s", 1e12),
        "upsilon": (lambda: native.rm_effective_collision_strengths(
                        E, omega, e_level, n_t, kT),
                    "hbm", 8.0 * M * P, 8000.0, "GB/s", 1e9),
        "group": (lambda: native.rm_group_collision_strengths(
                      omega, n_t, group, n_g),
                  "hbm", 8.0 * M * (P + Pg), 8000.0, "GB/s", 1e9),
    }
    res = {}
    for name, (fn, bound, units, peak, unit, scale) in calls.items():
        fn()
        torch.cuda.synchronize()
        native.rm_profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        k_ms, launches = native.rm_profile_query(name)
        native.rm_profile(False)
        k_ms /= max(1, launches)
        ach = units / (k_ms * 1e-3) / scale if k_ms > 0 else None
        res[name] = {"bound": bound, "achieved": ach, "peak": peak,
                     "unit": unit, "frac": ach / peak if ach else None,
                     "kernel_ms": k_ms, "call_ms": wall,
                     "algorithmic": units}
        note("postproc %s: kernel %.3f ms, call %.3f ms" % (name, k_ms, wall))
    res["setup"] = {"fwhm_meV": 100.0, "kT_Ry": [float(x) for x in kT],
                    "n_group": n_g, "transitions": P}
    del out
    return res


PHOTO_SHAPES = {
    # the paper's Table 1: B II, 409,600 energies in 149.70 s on 8192 Cray
    # XE6 cores; Table 2: Ca II, 6,000 energies in 108.23 s on 6000 Cray XE6
    # (Hopper) cores (both modules also damp resonances and read files)
    "b2": ("photo_b2", 409600 / 149.70, "8192 Cray XE6 cores (Table 1)"),
    "ca2": ("photo_ca2", 6000 / 108.2344, "6000 Cray XE6 cores (Table 2)"),
}


def photo_leg(native, torch, oracle, workloads, steps, warmup, count,
              shape="b2", n_check=4, damped=False):
    """Photoionization on the B II (Table 1: 400 channels, 409,600 energies)
    or Ca II (Table 2: 1815 channels, 6,000 energies) shape of the paper:
    `count` energies spread evenly over the mesh, timed like the headline;
    sigma checked against the oracle on `n_check` of them.  damped: with
    radiative widths (workloads.radiative_widths, seed 65) on the poles."""
    gen, paper_rate, paper_hw = PHOTO_SHAPES[shape]
    w, d, e0 = getattr(workloads, gen)()
    stride = max(1, w.mesh.size // count)
    Em = w.mesh[::stride][:count]
    h = native.load_symmetry(w.syms[0])
    native.rm_load_dipoles(h, d)
    opts = None
    if damped:
        G = workloads.radiative_widths(w.syms[0].n_poles, 65)
        native.rm_load_widths(h, G)
        opts = native.make_opts(flags=native.RM_FLAG_RADIATION_DAMPING)
    E = torch.as_tensor(Em, dtype=torch.float64, device="cuda:0")
    sig = torch.empty_like(E)
    st = torch.empty(E.shape, dtype=torch.int32, device=E.device)
    for _ in range(warmup):
        native.rm_photoionization([h], E, e0, opts, sigma=sig, status=st)
    torch.cuda.synchronize()
    native.rm_profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        native.rm_photoionization([h], E, e0, opts, sigma=sig, status=st)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    stage = {k: native.rm_profile_query(k)[0] / steps
             for k in ("polesum", "match")}
    native.rm_profile(False)
    idx = workloads.sample_indices(Em.size, n_check, seed=3)
    if damped:
        ref = oracle.photoionization_damped([w.syms[0].as_dict()], [d], [G],
                                            Em[idx], e0)
    else:
        ref = oracle.photoionization([w.syms[0].as_dict()], [d], Em[idx], e0)
    got = sig.cpu().numpy()[idx]
    err = float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))
    h.free()
    note("photoionization %s%s: %.1f ms for %d energies, err %.2e"
         % (w.name, " damped" if damped else "", ms, Em.size, err))
    return {"workload": w.name + ("+radiation damping" if damped else ""),
            "energies_timed": int(Em.size),
            "sample": "every %d-th energy of the %d-point mesh"
                      % (stride, w.mesh.size),
            "value": Em.size / (ms * 1e-3), "unit": "energies/s",
            "ms_per_step": ms, "steps": steps, "stage_ms_per_step": stage,
            "max_rel_err_sigma": err, "err_sample": int(idx.size),
            "paper_context": {"energies_per_s": paper_rate,
                              "hardware": paper_hw,
                              "ratio": Em.size / (ms * 1e-3) / paper_rate}}


def outer_leg(native, torch, oracle, workloads, steps, warmup, count,
              n_sec=20, width=20.0, w=None, gl_terms=0):
    """The headline symmetry (or the workload w) with the outer-region
    propagation switched on (dipole and quadrupole coupling, A = a + width,
    n_sec sectors; with gl_terms > 0 matched at A to the asymptotic
    expansion): `count` energies spread over the mesh, Omega checked against
    the oracle on 3."""
    from oracle import outer
    w = workloads.config2() if w is None else w
    sym = w.syms[0]
    beta = workloads.outer_coupling(sym.n)
    A = sym.a + width
    stride = max(1, w.mesh.size // count)
    Em = w.mesh[::stride][:count]
    h = native.load_symmetry(sym)
    t0 = time.perf_counter()
    native.rm_set_propagation(h, A, n_sec, beta)
    if gl_terms:
        native.rm_set_gailitis(h, gl_terms)
    setup = time.perf_counter() - t0
    E = torch.as_tensor(Em, dtype=torch.float64, device="cuda:0")
    P = w.n_target * (w.n_target + 1) // 2
    om = torch.empty((Em.size, P), dtype=torch.float64, device=E.device)
    st = torch.empty(E.shape, dtype=torch.int32, device=E.device)
    opts = native.make_opts()
    for _ in range(warmup):
        native.rm_sweep_energies([h], w.n_target, E, opts, om, st)
    torch.cuda.synchronize()
    native.rm_profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        native.rm_sweep_energies([h], w.n_target, E, opts, om, st)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    stage = {k: native.rm_profile_query(k)[0] / steps
             for k in ("polesum", "propagate", "match")}
    native.rm_profile(False)
    idx = workloads.sample_indices(Em.size, 3, seed=4)
    prop = {"A": A, "n_sec": n_sec, "beta": beta, "gailitis_terms": gl_terms}
    ref = outer.sweep_propagated(sym.as_dict(), prop, Em[idx], w.n_target)
    flagged = float(((st.cpu().numpy() & native.RM_E_ASYM_NOCONV) != 0).mean())
    got = om.cpu().numpy()[idx]
    err = float((np.abs(got - ref).max(axis=1)
                 / np.maximum(np.abs(ref).max(axis=1), 1e-300)).max())
    h.free()
    n = sym.n
    # per energy: per sector X O and O^T (X O) (2 n^3 each), the LU of the
    # sector system (2 n^3 / 3) and its n right-hand sides (2 n^3); the final
    # basis change (4 n^3)
    flops = Em.size * (n_sec * (4.0 + 2.0 / 3.0 + 2.0) + 4.0) * n ** 3
    ach = flops / (stage["propagate"] * 1e-3) / 1e12 if stage["propagate"] else None
    note("outer propagation%s: %.1f ms for %d energies (propagation %.1f ms), "
         "err %.2e" % (" + expansion" if gl_terms else "", ms, Em.size,
                       stage["propagate"], err))
    res = {"workload": w.name + "+outer(A=a+%g, %d sectors, lmax 2%s)"
                        % (width, n_sec,
                           ", expansion %d terms" % gl_terms if gl_terms else ""),
            "energies_timed": int(Em.size), "value": Em.size / (ms * 1e-3),
            "unit": "energies/s", "ms_per_step": ms,
            "stage_ms_per_step": stage, "setup_s": setup,
            "max_rel_err_omega": err, "err_sample": int(idx.size),
            "propagation_roofline": {"bound": "mfma", "achieved": ach,
                                     "peak": 78.6, "unit": "TFLOP/s",
                                     "frac": ach / 78.6 if ach else None,
                                     "flops_per_step": flops}}
    if gl_terms:
        res["asym_noconv_fraction"] = flagged
        res["propagation_roofline"]["note"] = (
            "flops count the sectors only; the stage also runs the expansion")
    return res


def inner_leg(native, oracle, workloads, steps, n_basis, no_cpu):
    """The inner-region eigen-solve that supplies the poles: a model of 8
    channels x n_basis sine functions (D = 8 n_basis), all eigenpairs on the
    device; eigenvalues checked against the oracle within the backward-error
    budget 8 (D + Q) eps S, S the spectrum's scale."""
    m = workloads.inner_model()
    n = m["e_thr"].size
    D = n * n_basis
    Q = n_basis + 48
    native.rm_inner_region(m, n_basis)          # warm-up (code objects)
    native.rm_profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        E, w, sweeps, rot = native.rm_inner_region(m, n_basis)
    s_per = (time.perf_counter() - t0) / steps
    jac_ms, jac_n = native.rm_profile_query("jacobi")
    asm_ms, _ = native.rm_profile_query("assemble")
    native.rm_profile(False)
    jac_ms /= steps
    asm_ms /= steps
    Dp = (D + 31) // 32 * 32              # 16-column blocks, an even number
    launches = sweeps * (Dp // 16 - 1)    # round-robin steps over the blocks
    # per step the Gram kernels read every column of A once; a rotated block
    # pair reads and writes its 32 columns of A and of V
    bytes_solve = launches * 8.0 * Dp * Dp + rot * 4.0 * 32 * 8 * Dp
    ach = bytes_solve / (jac_ms * 1e-3) / 1e9 if jac_ms else None
    t0 = time.perf_counter()
    Eo, wo = oracle.inner.inner_region(m, n_basis)
    cpu_s = time.perf_counter() - t0
    S = max(float(np.abs(Eo).max()), 1.0)
    eta = 8.0 * (D + Q) * np.finfo(float).eps * S
    ratio = float(np.abs(E - Eo).max() / eta)
    note("inner region D=%d: %.3f s per solve (%d sweeps, Jacobi %.1f ms, "
         "assembly %.1f ms), eigenvalue error / budget %.2e"
         % (D, s_per, sweeps, jac_ms, asm_ms, ratio))
    out = {"workload": "model inner region, %d channels x %d sine functions "
                       "(D = %d), a = %g" % (n, n_basis, D, m["a"]),
           "value": 1.0 / s_per, "unit": "solves/s", "s_per_solve": s_per,
           "sweeps": int(sweeps), "rotations": int(rot),
           "jacobi_ms": jac_ms, "assembly_ms": asm_ms,
           "jacobi_steps": int(launches),
           "eigenvalue_err_over_budget": ratio,
           "jacobi_roofline": {"bound": "hbm", "achieved": ach, "peak": 8000.0,
                               "unit": "GB/s",
                               "frac": ach / 8000.0 if ach else None,
                               "bytes_per_solve": bytes_solve}}
    # eight symmetries of D = 1024 (4 channels x 256), one by one and batched
    models = [workloads.inner_model(n=4, seed=30 + b) for b in range(8)]
    native.rm_inner_region_batch(models[:2], 256)
    t0 = time.perf_counter()
    for mb in models:
        native.rm_inner_region(mb, 256)
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    native.rm_inner_region_batch(models, 256)
    t_bat = time.perf_counter() - t0
    out["batch_8x_D1024"] = {"s_one_by_one": t_seq, "s_batched": t_bat,
                             "speedup": t_seq / t_bat}
    # the D = 4096 model's poles swept like the headline symmetry: 20000
    # energies in [0, 20] (all 8 channels their own target level)
    import torch
    h = native.rm_load_poles(E, w, m["a"], m["e_thr"], m["l"], m["z"], 1.0)
    Em = workloads.uniform_mesh(0.0, 20.0, 20000)
    Et = torch.as_tensor(Em, dtype=torch.float64, device="cuda:0")
    om, st = native.rm_sweep_energies([h], n, Et)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    om, st = native.rm_sweep_energies([h], n, Et)
    torch.cuda.synchronize()
    t_sw = time.perf_counter() - t0
    idx = workloads.sample_indices(Em.size, 4, seed=5)
    sym = {"E_pole": E, "w": w, "a": m["a"], "e_thr": m["e_thr"], "l": m["l"],
           "z": m["z"], "g": 1.0}
    ref = oracle.sweep(sym, Em[idx], n_target=n)["omega"]
    got = om.cpu().numpy()[idx]
    sw_err = float((np.abs(got - ref).max(axis=1)
                    / np.maximum(np.abs(ref).max(axis=1), 1e-300)).max())
    h.free()
    out["sweep_over_these_poles"] = {"energies": int(Em.size),
                                     "value": Em.size / t_sw,
                                     "unit": "energies/s",
                                     "max_rel_err_omega": sw_err,
                                     "err_sample": int(idx.size)}
    note("inner region: 8 x D=1024 %.3f s one by one, %.3f s batched; sweep "
         "over the D=4096 poles %.0f energies/s (err %.1e)"
         % (t_seq, t_bat, Em.size / t_sw, sw_err))
    if not no_cpu:
        out["cpu_baseline"] = {"value": 1.0 / cpu_s, "unit": "solves/s",
                               "cores": blas_threads(), "kind": "oracle",
                               "sample": "one full solve of the same model "
                                         "(quadrature, assembly, LAPACK eigh)"}
    return out


def c5_leg(n_train, workers, log):
    """The learned adaptive mesh at full size: trained on seeds 1000 ..
    1000 + n_train - 1 of the narrow-resonance generator (200 channels,
    8000 + 50 poles; one 1 Ry sub-window of the 2e-5 Ry fine spacing per
    seed), judged on seed 3000 against its 1e6-point uniform FP64 sweep on
    [0, 20] Ry, 1e5 adaptive points; truth resonances measured by the
    oracle from the slope of the eigenphase sum."""
    from oracle import resonance
    from paper_1403_5524_amd import adaptive

    def truth(sym, nominal):
        return resonance.measure_list(sym.as_dict(), nominal, workers=workers)
    t0 = time.perf_counter()
    res = adaptive.run_experiment(train_seeds=list(range(1000, 1000 + n_train)),
                                  test_seed=3000, truth_fn=truth, log=log)
    res["seconds"] = time.perf_counter() - t0
    res.pop("train_loss", None)
    return res


def table3_leg(native, torch, oracle, workloads):
    """The FP64 pole sum (rm_rmatrix) on the ten shapes of the paper's
    Table 3: enough energies per shape to fill the GPU (4096, fewer for the
    largest shapes, at least 256), kernel time from the pole-sum stage,
    R checked against the oracle on one energy for n <= 400."""
    rows = []
    for n, m in workloads.TABLE3_SHAPES:
        M = int(min(4096, max(256, 2e13 / (n * (n + 1.0) * m))))
        sym, mesh = workloads.table3_symmetry(n, m, M)
        h = native.load_symmetry(sym)
        E = torch.as_tensor(mesh, dtype=torch.float64, device="cuda:0")
        native.rm_rmatrix(h, E[:64])                # warm-up
        torch.cuda.synchronize()
        native.rm_profile(True)
        R = native.rm_rmatrix(h, E)
        torch.cuda.synchronize()
        ms, _ = native.rm_profile_query("polesum")
        native.rm_profile(False)
        err = None
        if n <= 400:
            k = M // 3
            ref = oracle.r_matrix(sym.E_pole, sym.w, sym.a, mesh[k:k + 1])[0]
            err = float(np.abs(R[k].cpu().numpy() - ref).max() / np.abs(ref).max())
        del R
        h.free()
        flops = n * (n + 1.0) * m * M
        tf = flops / (ms * 1e-3) / 1e12
        rows.append({"n": n, "m": m, "energies": M, "ms": ms,
                     "ms_per_multiply": ms / M, "tflops": tf,
                     "frac": tf / PEAK["fp64"], "max_rel_err_R": err})
        note("table 3 shape %d x %d: %d energies in %.1f ms, %.1f TFLOP/s"
             % (n, m, M, ms, tf))
    return {"rows": rows,
            "note": "FP64 pole sum only; flops counted as n(n+1)m per energy "
                    "(upper triangle); the paper's Table 3 times (TITAN, unit "
                    "ambiguous) are context only"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp64", choices=sorted(PREC_CODE))
    ap.add_argument("--M", type=int, default=100000)
    ap.add_argument("--err-sample", type=int, default=32)
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--also", default="bf16x3,fp32,fp32/s32",
                    help="comma-separated precisions also timed on the same "
                         "workload (reported under other_precisions); a "
                         "\"/s32\" suffix also factors the matching solve "
                         "in FP32 with FP64 refinement")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4"],
                    help="c2 is the headline workload; c3 (40 symmetries) "
                         "and c4 (1500 channels) time a prefix of their mesh")
    ap.add_argument("--graph", action="store_true",
                    help="also time replays of a hipGraph-captured plan")
    ap.add_argument("--no-postproc", action="store_true",
                    help="skip timing the post-processing of Omega")
    ap.add_argument("--outer-M", type=int, default=2048,
                    help="energies of the outer-region propagation leg; "
                         "0 skips it")
    ap.add_argument("--inner-N", type=int, default=512,
                    help="sine functions per channel of the inner-region "
                         "leg (8 channels); 0 skips it")
    ap.add_argument("--table3", action="store_true",
                    help="also time the FP64 pole sum on the ten shapes of "
                         "the paper's Table 3 (reported under table3)")
    ap.add_argument("--photo-ca-M", type=int, default=2048,
                    help="energies of the photoionization leg on the Ca II "
                         "shape (1815 channels, 6000 energies); 0 skips it")
    ap.add_argument("--c5-train", type=int, default=32,
                    help="training seeds of the learned-mesh leg (full-size "
                         "1e6-point judge, 1e5 adaptive points); 0 skips it")
    ap.add_argument("--photo-M", type=int, default=8192,
                    help="energies of the photoionization leg (B II shape); "
                         "0 skips it")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: every energy is independent, so "
              "more GPUs would split the mesh (see the sharding note in the "
              "design document); no multi-GPU run is provided.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import oracle
    from paper_1403_5524_amd import native, workloads

    dev = torch.device("cuda:0")
    if args.workload == "c2":
        w = workloads.config2(M=args.M)
    elif args.workload == "c3":
        w = workloads.config3()
        w.mesh = w.mesh[:: max(1, w.mesh.size // args.M)][:args.M]
    else:
        w = workloads.config4()
        w.mesh = w.mesh[:: max(1, w.mesh.size // args.M)][:args.M]
    sym = w.syms[0]
    n_t = w.n_target
    nh = sym.n_poles
    n = sym.n
    M = w.mesh.size
    P = n_t * (n_t + 1) // 2
    note("loading %s (%d energies timed)" % (w.name, M))
    hs = [native.load_symmetry(s) for s in w.syms]
    E = torch.as_tensor(w.mesh, dtype=torch.float64, device=dev)
    omega = torch.empty((M, P), dtype=torch.float64, device=dev)
    status = torch.empty((M,), dtype=torch.int32, device=dev)

    pairs = 0.0
    flops_step = 0.0
    mflops_step = 0.0
    mflops_exec = 0.0
    for s in w.syms:
        n_open = np.searchsorted(np.sort(s.e_thr), w.mesh, side="left")
        pairs += float((n_open * (n_open + 1) // 2).sum())
        flops_step += float(s.n) * (s.n + 1) * s.n_poles * M   # symmetric
        mflops_step += match_flops(s.n, n_open)
        mflops_exec += match_flops_executed(s.n, n_open)
    cpu_rec = None
    if not args.no_cpu and len(w.syms) == 1:
        # the oracle's timed sample doubles as the error sample
        note("cpu baseline on %d energies" % args.cpu_sample)
        cpu_rec, idx, ref = cpu_baseline(sym, w.mesh, args.cpu_sample)
    else:
        idx = workloads.sample_indices(M, args.err_sample, seed=7)
        ref = None
        for s in w.syms:
            r = oracle.sweep(s.as_dict(), w.mesh[idx], n_target=n_t)["omega"]
            ref = r if ref is None else ref + r
    idx_dev = torch.as_tensor(idx, device=dev)

    def run(name, graph, steps=None, warmup=None):
        """Warm up, time `steps` sweeps at one precision, check Omega.
        `name` is a pole-sum precision, optionally with "/s32": the
        matching solve factored in FP32 and refined in FP64."""
        steps = args.steps if steps is None else steps
        warmup = args.warmup if warmup is None else warmup
        prec, _, solve = name.partition("/")
        opts = native.make_opts(prec=PREC_CODE[prec],
                                solve_fp32=1 if solve == "s32" else 0)
        for i in range(warmup):
            native.rm_sweep_energies(hs, n_t, E, opts, omega, status)
            torch.cuda.synchronize()
            note("%s warmup %d done" % (name, i + 1))
        native.rm_profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            native.rm_sweep_energies(hs, n_t, E, opts, omega, status)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        native.rm_profile(False)
        ms = (t1 - t0) * 1e3 / steps
        note("%s: timed %d steps: %.2f ms/step" % (name, steps, ms))
        stage = {k: native.rm_profile_query(k) for k in ("polesum", "match")}
        graph_ms = None
        if graph:
            plan = native.Plan(hs, n_t, E, opts, omega, status)
            plan.execute()
            torch.cuda.synchronize()
            g0 = time.perf_counter()
            for i in range(steps):
                plan.execute()
            torch.cuda.synchronize()
            graph_ms = (time.perf_counter() - g0) * 1e3 / steps
            plan.free()
            note("%s: graph replays %.2f ms/step" % (name, graph_ms))
        got = omega[idx_dev].cpu().numpy()
        err, err_el = omega_errors(got, ref)
        st = status.cpu().numpy()
        note("%s: max rel err of Omega on %d sampled energies: %.3e "
             "normwise, %.3e elementwise" % (name, idx.size, err, err_el))
        kernels = {}
        for key, flops, peak, stg, tkey in (
                ("polesum_%s" % prec, flops_step, PEAK[prec], "polesum",
                 "polesum_%s" % prec),
                ("match_kernel", mflops_step, PEAK["fp64"], "match",
                 "match_kernel")):
            ms_tot, launches = stage[stg]
            lp = launches / steps if launches else 0
            ach = (flops * steps / (ms_tot * 1e-3) / 1e12
                   if ms_tot > 0 else None)
            traffic = measured_traffic(tkey, M / lp) if (tkey and lp) else None
            kernels[key] = {
                "bound": "mfma", "kernel": key, "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak if ach else None,
                "traffic": traffic,
                "flops_per_launch": flops / lp if lp else None,
                "avg_launch_ms": ms_tot / launches if launches else None,
                "ms_per_step": ms_tot / steps}
        mk = kernels["match_kernel"]
        if mk["achieved"]:
            # the flops the kernel runs: its LU does 2n^3/3 where the minimal
            # count has the n^3/3 of a symmetric factorisation, its T step
            # 3 n_o^3 where the minimal count has 16 n_o^3/3
            mk["achieved_executed_flops"] = mk["achieved"] * mflops_exec / mflops_step
            mk["flops_note"] = ("achieved counts n^3/3 + 2 n^2 n_o + 16 n_o^3/3 "
                                "per energy; achieved_executed_flops counts "
                                "2 n^3/3 + 2 n^2 n_o + 3 n_o^3, what the "
                                "kernel runs")
        return {"ms": ms, "err": err, "err_el": err_el,
                "flagged": int((st != 0).sum()),
                "stage": {k: v[0] / args.steps for k, v in stage.items()},
                "kernels": kernels, "graph_ms": graph_ms}

    head = run(args.prec, args.graph)
    # combined roofline of a step: the pole sums at the MFMA peak of their
    # precision, the dense FP64 step at the FP64 peak, the Omega writes and
    # energy reads at the HBM bandwidth
    t_roof = (flops_step / (PEAK[args.prec] * 1e12)
              + mflops_step / (PEAK["fp64"] * 1e12)
              + (8.0 * P * M + 8.0 * M) / 8e12)
    combined = {"t_roof_ms": t_roof * 1e3, "t_ms": head["ms"],
                "frac": t_roof * 1e3 / head["ms"],
                "terms_ms": {"polesum": flops_step / (PEAK[args.prec] * 1e9),
                             "dense": mflops_step / (PEAK["fp64"] * 1e9),
                             "hbm": (8.0 * P * M + 8.0 * M) / 8e9}}
    gemm_ceiling = (library_gemm_ceiling(torch, sym, w.mesh)
                    if len(w.syms) == 1 else None)
    post = None
    if not args.no_postproc and len(w.syms) == 1 and sym.target is None:
        # every channel its own target level: level energies are thresholds
        post = postproc_leg(native, torch, E, omega, w.mesh, sym.e_thr, n_t,
                            max(1, args.steps))
    others = {}
    for prec in [p for p in args.also.split(",") if p and p != args.prec]:
        r = run(prec, False, steps=min(args.steps, 5),
                warmup=min(args.warmup, 1))
        others[prec] = {
            "value": M / (r["ms"] * 1e-3), "ms_per_step": r["ms"],
            "max_rel_err_omega": r["err"],
            "max_rel_err_omega_normwise": r["err"],
            "max_rel_err_omega_elementwise": r["err_el"],
            "status_flagged": r["flagged"],
            "speedup_over_%s" % args.prec: head["ms"] / r["ms"],
            "stage_ms_per_step": r["stage"], "kernels": r["kernels"]}
    outer_res = outer_gl_res = None
    if args.outer_M > 0:
        outer_res = outer_leg(native, torch, oracle, workloads, args.steps,
                              args.warmup, args.outer_M)
        # matched to the asymptotic expansion at A = 200: a target of 10
        # levels 0.5 Ry apart, propagated through 90 sectors of 2 a0
        outer_gl_res = outer_leg(native, torch, oracle, workloads, args.steps,
                                 args.warmup, args.outer_M, n_sec=90,
                                 width=180.0,
                                 w=workloads.outer_levels(M=args.outer_M),
                                 gl_terms=40)
    photo = None
    if args.photo_M > 0:
        photo = photo_leg(native, torch, oracle, workloads, args.steps,
                          args.warmup, args.photo_M)
    photo_damped = None
    if args.photo_M > 0:
        photo_damped = photo_leg(native, torch, oracle, workloads,
                                 min(args.steps, 3), min(args.warmup, 1),
                                 args.photo_M // 4, n_check=3, damped=True)
    photo_ca = None
    if args.photo_ca_M > 0:
        # one untimed-warmup-free step: the headline run has loaded the code
        photo_ca = photo_leg(native, torch, oracle, workloads, 1, 0,
                             args.photo_ca_M, shape="ca2", n_check=2)
    table3 = table3_leg(native, torch, oracle, workloads) if args.table3 else None
    c5 = None
    if args.c5_train > 0:
        c5 = c5_leg(args.c5_train, max(1, min(16, (os.cpu_count() or 2) - 1)),
                    note)
    inner_res = None
    if args.inner_N > 0:
        inner_res = inner_leg(native, oracle, workloads, max(1, min(args.steps, 2)),
                              args.inner_N, args.no_cpu)
    ms = head["ms"]
    dom = max(head["kernels"].values(), key=lambda k: k["ms_per_step"])
    roof = dict(dom)
    graph_ms = head["graph_ms"]
    out = {
        "metric": "energy points/sec (K->Omega) at n=200 ch, N_H=8000; "
                  "max rel err of Omega vs FP64 oracle",
        "value": M / (ms * 1e-3),
        "unit": "energies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f64+%s" % args.prec,
        "data": "synthetic (seeded poles/amplitudes, C2 shape)",
        "config": {"workload": w.name, "n_sym": len(w.syms), "n_chan": n,
                   "n_poles": nh, "energies": M,
                   "mesh_Ry": [float(w.mesh_spec[0]), float(w.mesh_spec[1])],
                   "precision": args.prec},
        "max_rel_err_omega": head["err"],
        "max_rel_err_omega_normwise": head["err"],
        "max_rel_err_omega_elementwise": head["err_el"],
        "err_sample": int(idx.size),
        "err_sample_kind": ("the cpu_baseline's oracle energies"
                            if cpu_rec is not None else
                            "seeded sample of mesh energies"),
        "omega_per_s": pairs / (ms * 1e-3),
        "status_flagged": head["flagged"],
        "stage_ms_per_step": head["stage"],
        "kernels": head["kernels"],
        "graph_ms_per_step": graph_ms,
        "graph_value": (M / (graph_ms * 1e-3)) if graph_ms else None,
        "roofline": roof,
        "combined_roofline": combined,
        "library_gemm_ceiling": gemm_ceiling,
        "other_precisions": others,
        "postproc": post,
        "photoionization": photo,
        "photoionization_damped": photo_damped,
        "photoionization_ca2": photo_ca,
        "outer_propagation": outer_res,
        "outer_expansion": outer_gl_res,
        "inner_region": inner_res,
        "learned_mesh": c5,
        "table3": table3,
    }
    if cpu_rec is not None:
        out["cpu_baseline"] = cpu_rec
        out["cpu_baseline_1thread"] = cpu_baseline_1thread(
            sym, w.mesh, max(1, args.cpu_sample // 32))
    for h in hs:
        h.free()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
