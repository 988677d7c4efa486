"""Resonance positions and widths from the eigenphase sum (FP64 oracle).

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see the package docstring).

Used to measure the truth list of the learned-mesh experiment: the paper
asks for fine meshes because of narrow resonances (Sec. 3) and gives no
recipe for locating them.  Read as standard R-matrix practice: across an
isolated resonance the eigenphase sum sum_i delta_i(E), delta_i =
atan(eig_i K(E)), rises by pi with the Breit-Wigner profile
atan(2 (E - E_r) / Gamma), so its slope peaks at E_r with the value
2 / Gamma.  The measurement scans the sum on a local grid (unwrapped across
branches of atan), takes the point of largest slope, refines it with the
parabola through its neighbours, converts the largest difference quotient
to a width (exactly, for the arctan profile, whatever the grid step), and
repeats on a grid a few widths wide.
"""
import numpy as np

from .rmatrix import r_matrix, channel_data, k_matrix, eigenphases


def eigenphase_sum(sym, E):
    """sum_i atan(eig_i K(E)) at each energy of E (open-open K)."""
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    a = float(sym["a"])
    cd = channel_data(E, sym["e_thr"], sym["l"], sym["z"], a)
    R = r_matrix(sym["E_pole"], sym["w"], a, E)
    out = np.empty(E.size)
    for m in range(E.size):
        K, P = k_matrix(R[m], a, cd["open"][m], cd["s"][m], cd["c"][m],
                        cd["sp"][m], cd["cp"][m], cd["L"][m])
        out[m] = eigenphases(K).sum() if P.size else 0.0
    return out


def _peak_slope(E, d):
    """Energy and value of the largest slope of d(E) on a uniform grid,
    refined by the parabola through the neighbouring slopes."""
    # the sum is defined modulo pi per eigenphase crossing atan's branch
    d = np.unwrap(2.0 * d) / 2.0
    h = E[1] - E[0]
    s = np.diff(d) / h
    mid = 0.5 * (E[1:] + E[:-1])
    i = int(np.argmax(s))
    if 0 < i < s.size - 1:
        y0, y1, y2 = s[i - 1], s[i], s[i + 1]
        den = y0 - 2.0 * y1 + y2
        t = 0.5 * (y0 - y2) / den if den != 0.0 else 0.0
        t = min(max(t, -0.5), 0.5)
        return mid[i] + t * h, y1 - 0.25 * (y0 - y2) * t
    return mid[i], s[i]


def _width(smax, h):
    """Gamma from the largest difference quotient smax on a grid of step h:
    for atan(2 (E - E_r) / Gamma) the centred quotient at E_r is
    (2 / h) atan(h / Gamma), so Gamma = h / tan(h smax / 2) (2 / smax when
    h << Gamma)."""
    x = 0.5 * h * smax
    return h / np.tan(x) if 0.0 < x < 0.5 * np.pi else 2.0 / smax


def measure_resonance(sym, E_guess, span, n=40, levels=14, refine=2):
    """(E_r, Gamma) of the resonance near E_guess.

    Grids of n points centred on E_guess shrink by 4 per level from
    +- span until the eigenphase sum rises by more than pi/2 across the
    grid with its steepest point in the central half: the resonance is then
    inside and resolved (below that, a rise of pi between two grid points is
    invisible modulo pi; off centre, it belongs to a wider neighbour).  Its slope peak
    gives (E_r, 2 / slope), refined on grids of +- 4 Gamma around it.  n is
    even, so a grid centred on a pole energy never evaluates on it.  Returns
    NaNs if no level shows the rise."""
    n += n % 2
    half = float(span)
    for _ in range(levels):
        E = np.linspace(E_guess - half, E_guess + half, n)
        d = eigenphase_sum(sym, E)
        if not np.all(np.isfinite(d)):
            return float("nan"), float("nan")
        du = np.unwrap(2.0 * d) / 2.0
        Er, smax = _peak_slope(E, d)
        # a rise of over pi/2 whose steepest point is in the central half:
        # the resonance at E_guess, not a wider neighbour at the edge
        if du[-1] - du[0] > 0.5 * np.pi and abs(Er - E_guess) < 0.5 * half:
            G = _width(smax, E[1] - E[0])
            for _ in range(refine):
                E = np.linspace(Er - 4.0 * G, Er + 4.0 * G, n)
                Er, smax = _peak_slope(E, eigenphase_sum(sym, E))
                G = _width(smax, E[1] - E[0])
            return float(Er), float(G)
        half /= 4.0
    return float("nan"), float("nan")


def _measure_one(args):
    sym, Er, span = args
    return measure_resonance(sym, Er, span)


def measure_list(sym, nominal, span_factor=30.0, workers=1):
    """Measure every resonance of a nominal (E, width) list: each scan
    starts at E over +- span_factor * width.  workers > 1 spreads the
    resonances over that many processes (one BLAS thread each)."""
    jobs = [(sym, float(E), span_factor * float(G)) for E, G in nominal]
    if workers <= 1:
        return [_measure_one(j) for j in jobs]
    import multiprocessing as mp
    import os
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                          "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            return pool.map(_measure_one, jobs)
    finally:
        for k, v in env.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
