"""Shared helpers for the GPU parity tests (HIP path vs the CPU oracle)."""
import sys

import numpy as np

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def omega_normwise_err(om_gpu, om_ref):
    """Max over energies of max|dOmega| / max|Omega_ref| (energies with
    Omega_ref == 0 use an absolute 1e-300 floor)."""
    om_gpu = np.asarray(om_gpu)
    om_ref = np.asarray(om_ref)
    num = np.abs(om_gpu - om_ref).max(axis=1)
    den = np.maximum(np.abs(om_ref).max(axis=1), 1e-300)
    return float((num / den).max()), num, den


def omega_elementwise_err(om_gpu, om_ref, floor=1e-8):
    """Max of |dOmega| / |Omega_ref| over every transition whose reference
    is at least `floor` times the largest value of its energy's row."""
    om_gpu = np.asarray(om_gpu)
    om_ref = np.asarray(om_ref)
    row = np.abs(om_ref).max(axis=1, keepdims=True)
    big = (np.abs(om_ref) >= floor * row) & (row > 0)
    rel = np.abs(om_gpu - om_ref) / np.maximum(np.abs(om_ref), 1e-300)
    return float(np.where(big, rel, 0.0).max()) if om_ref.size else 0.0


def oracle_channel_table(sym, E):
    """Oracle channel functions laid out like rm_channel_functions."""
    cd = oracle.channel_data(E, sym["e_thr"], sym["l"], sym["z"], sym["a"])
    a = float(sym["a"])
    m, n = cd["open"].shape
    out = np.zeros((m, n, 4))
    op = cd["open"]
    out[..., 0] = np.where(op, cd["s"], 0.0)
    out[..., 1] = np.where(op, cd["c"], 0.0)
    out[..., 2] = np.where(op, a * cd["sp"], 0.0)
    out[..., 3] = np.where(op, a * cd["cp"], 0.0)
    L = np.where(op, 0.0, cd["L"])
    nrm = np.hypot(1.0, L)
    out[..., 0] = np.where(op, out[..., 0], 1.0 / nrm)
    out[..., 1] = np.where(op, out[..., 1], L / nrm)
    return out, op


def oracle_sweep_multi(syms, E, n_target):
    """Sum of per-symmetry oracle Omega (shared target levels)."""
    tot = None
    st = np.zeros(len(E), dtype=np.int32)
    for s in syms:
        d = s.as_dict() if hasattr(s, "as_dict") else s
        r = oracle.sweep(d, E, n_target=n_target)
        tot = r["omega"] if tot is None else tot + r["omega"]
        st |= r["status"]
    return tot, st
