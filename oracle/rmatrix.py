"""R-matrix outer-region sweep, one energy at a time, in FP64 (oracle).

TEST INFRASTRUCTURE: only tests/, smoke() and bench.py's cpu_baseline may use it.

Units: Rydberg energies, Bohr radii.  A symmetry is a mapping with keys

    E_pole [N_H]      poles E_k, ascending
    w      [n, N_H]   surface amplitudes w_ik
    a                 boundary radius
    e_thr  [n]        channel thresholds e_i
    l      [n]        channel orbital angular momenta
    target [n] / None target level of each channel (None: channel i -> i)
    z                 residual charge
    g                 statistical weight of the symmetry (2J+1)

Readings of the paper used here (Sec. 6, Eq. 1-2 give only the pole sum, with
an index typo and no prefactor; the rest is standard R-matrix theory):

* R_ij(E) = (1/2a) sum_k w_ik w_jk / (E_k - E).  Eq. 1 prints
  sum_k W_ik W_kj / (E - E_k); the sign and 1/(2a) are fixed by requiring the
  Bloch-operator definition u(a) = a R u'(a) (Bloch constant b = 0) in Rydberg
  units with amplitudes w = sqrt(2) u_k(a).
* Matching at r = a to s = k^-1/2 F, c = k^-1/2 G (open) and the decaying
  Whittaker function (closed), written as one linear system for K and the
  closed-channel coefficients (no division by any channel function).
* T = 2iK (1 - iK)^-1, S = 1 + T.
* Omega(t, t') = sum over open channels i of target t and j of target t' of
  (g/2)|T_ij|^2, stored as the packed upper triangle t <= t'.
"""
import numpy as np

from .coulomb import open_channel_functions, closed_channel_logderiv

STATUS_NO_OPEN = 1


def r_matrix(E_pole, w, a, E):
    """Boundary R-matrix at each energy of ``E`` (Sec. 6, Eq. 1-2).

    Written as the paper's product R = X Y with X_ik = w_ik d_k,
    Y_kj = w_jk and d_k = 1/(E_k - E), times 1/(2a).  Returns [m, n, n].
    """
    E_pole = np.asarray(E_pole, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    out = np.empty((E.size, w.shape[0], w.shape[0]))
    for m, e in enumerate(E):
        d = 1.0 / (E_pole - e)
        X = w * d[None, :]
        out[m] = (X @ w.T) / (2.0 * a)
    return out


def channel_data(E, e_thr, l, z, a):
    """Open/closed split and boundary values of every channel at every energy.

    Returns a dict of [m, n] arrays: ``open`` (E > e_i, strict), and for open
    channels ``s, c, sp, cp`` (values and r-derivatives at r = a), for closed
    channels ``L`` = a W'(a)/W(a).  Entries of the other kind are NaN.
    """
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    e_thr = np.asarray(e_thr, dtype=np.float64)
    l = np.asarray(l, dtype=np.int64)
    m, n = E.size, e_thr.size
    diff = E[:, None] - e_thr[None, :]
    is_open = diff > 0.0
    ll = np.broadcast_to(l[None, :], (m, n))
    s = np.full((m, n), np.nan)
    c = np.full((m, n), np.nan)
    sp = np.full((m, n), np.nan)
    cp = np.full((m, n), np.nan)
    L = np.full((m, n), np.nan)
    if is_open.any():
        k = np.sqrt(diff[is_open])
        s[is_open], c[is_open], sp[is_open], cp[is_open] = \
            open_channel_functions(ll[is_open], z, k, a)
    cl = ~is_open
    if cl.any():
        phi = np.sqrt(-diff[cl])
        L[cl] = closed_channel_logderiv(ll[cl], z, phi, a)
    return {"open": is_open, "s": s, "c": c, "sp": sp, "cp": cp, "L": L}


def _closed_unit(L):
    """(W, a W') of a closed channel scaled to unit length: (1, L)/sqrt(1+L^2).

    Both components are returned; the second already includes the factor a.
    """
    nrm = np.hypot(1.0, L)
    return 1.0 / nrm, L / nrm


def k_matrix(R, a, open_mask, s, c, sp, cp, L):
    """Open-open K-matrix from the matching conditions at r = a.

    For each open channel j the solution vector u has open components
    s_i delta_ij + c_i K_ij and closed components e_i X_ij, with
    (e_i, a e_i') the closed-channel function scaled to unit length.  The
    R-matrix relation u(a) = R a u'(a) is one linear system in [K; X]:

        (D1 - R D2) [K; X] = R[:, P] diag(a s'_P) - [diag(s_P); 0]

    with D1 = diag(c_P, e_Q) and D2 = diag(a c'_P, a e'_Q), where for a
    closed channel (e, a e') = (1, L)/sqrt(1 + L^2) and L = a W'(a)/W(a).  Channels keep
    their own order; P is the ascending list of open channels.
    Returns (K [n_o, n_o], P).
    """
    P = np.nonzero(open_mask)[0]
    n = R.shape[0]
    if P.size == 0:
        return np.zeros((0, 0)), P
    d1 = np.empty(n)
    d2 = np.empty(n)
    d1[open_mask] = c[open_mask]
    d2[open_mask] = a * cp[open_mask]
    eq, aeqp = _closed_unit(L[~open_mask])
    d1[~open_mask] = eq
    d2[~open_mask] = aeqp
    A = np.diag(d1) - R * d2[None, :]
    B = R[:, P] * (a * sp[P])[None, :]
    B[P, np.arange(P.size)] -= s[P]
    Z = np.linalg.solve(A, B)
    return Z[P, :], P


def k_matrix_elimination(R, a, open_mask, s, c, sp, cp, L):
    """Same K by eliminating the closed channels first (cross-check only).

    With v = a u', closed rows give (diag(1/L) - R_QQ) v_Q = R_QP v_P, hence
    u_P = R' v_P with R' = R_PP + R_PQ (diag(1/L) - R_QQ)^-1 R_QP, and then
    (C - a R' C') K = a R' S' - S over the open channels alone.
    """
    P = np.nonzero(open_mask)[0]
    Q = np.nonzero(~open_mask)[0]
    if P.size == 0:
        return np.zeros((0, 0)), P
    Rp = R[np.ix_(P, P)].copy()
    if Q.size:
        Dq = np.diag(1.0 / L[Q]) - R[np.ix_(Q, Q)]
        Rp += R[np.ix_(P, Q)] @ np.linalg.solve(Dq, R[np.ix_(Q, P)])
    A = np.diag(c[P]) - a * Rp * cp[P][None, :]
    B = a * Rp * sp[P][None, :] - np.diag(s[P])
    return np.linalg.solve(A, B), P


def k_matrix_lambda(R, a, open_mask, s, c, sp, cp, L):
    """Same K through the inverse of Lambda - R (cross-check only).

    Lambda = diag(c/(a c')) on open channels and diag(1/L) on closed ones;
    K = -diag(s'/c') + (1/a) diag(1/c') [(Lambda - R)^-1]_PP diag(1/c'),
    which uses c s' - s c' = 1.
    """
    P = np.nonzero(open_mask)[0]
    if P.size == 0:
        return np.zeros((0, 0)), P
    lam = np.empty(R.shape[0])
    lam[open_mask] = c[open_mask] / (a * cp[open_mask])
    lam[~open_mask] = 1.0 / L[~open_mask]
    X = np.linalg.inv(np.diag(lam) - R)[np.ix_(P, P)]
    icp = 1.0 / cp[P]
    return -np.diag(sp[P] * icp) + (icp[:, None] * X * icp[None, :]) / a, P


def t_matrix(K):
    """T = 2iK (1 - iK)^-1, complex (K and (1 - iK)^-1 commute)."""
    n = K.shape[0]
    return np.linalg.solve(np.eye(n) - 1j * K, 2j * K.astype(np.complex128))


def s_matrix(K):
    """S = (1 + iK)(1 - iK)^-1 = 1 + T."""
    return np.eye(K.shape[0]) + t_matrix(K)


def eigenphases(K):
    """Eigenphases delta = arctan(eigenvalues of K)."""
    return np.arctan(np.linalg.eigvalsh(0.5 * (K + K.T)))


def omega_pair_index(t, u, n_target):
    """Position of target pair (t, u), t <= u, in the packed upper triangle.

    Row-major over t: (0,0), (0,1), ..., (0,N-1), (1,1), ...
    """
    return t * n_target - (t * (t - 1)) // 2 + (u - t)


def collision_strengths(T, P, target, n_target, g):
    """Packed Omega(t, t') = sum_{i in t, j in t', open} (g/2) |T_ij|^2.

    ``P`` lists the open channels that index T's rows/columns; ``target``
    maps channel -> target level (None: identity).  For t < t' each channel
    pair is counted once (i in t, j in t'); for t = t' all ordered pairs.
    """
    out = np.zeros(n_target * (n_target + 1) // 2)
    if len(P) == 0:
        return out
    tg = np.asarray(P) if target is None else np.asarray(target)[P]
    T2 = np.abs(T) ** 2
    for a_, ti in enumerate(tg):
        for b_, tj in enumerate(tg):
            if ti <= tj:
                out[omega_pair_index(int(ti), int(tj), n_target)] += \
                    0.5 * g * T2[a_, b_]
    return out


def sweep(sym, E, n_target=None, keep=()):
    """Omega(E) for one symmetry over a mesh: Eq. 1-2, matching, K, T, Omega.

    ``keep`` may contain "R", "K", "T" to also return those per energy.
    Returns dict with ``omega`` [m, n_target(n_target+1)/2], ``status`` [m]
    and the requested per-energy lists.
    """
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    n = len(sym["e_thr"])
    target = sym.get("target")
    if n_target is None:
        n_target = n if target is None else int(np.max(target)) + 1
    a = float(sym["a"])
    cd = channel_data(E, sym["e_thr"], sym["l"], sym["z"], a)
    R_all = r_matrix(sym["E_pole"], sym["w"], a, E)
    out = {"omega": np.zeros((E.size, n_target * (n_target + 1) // 2)),
           "status": np.zeros(E.size, dtype=np.int32)}
    for key in keep:
        out[key] = []
    for m in range(E.size):
        args = (cd["open"][m], cd["s"][m], cd["c"][m], cd["sp"][m],
                cd["cp"][m], cd["L"][m])
        K, P = k_matrix(R_all[m], a, *args)
        if P.size == 0:
            out["status"][m] |= STATUS_NO_OPEN
            T = np.zeros((0, 0), dtype=np.complex128)
        else:
            T = t_matrix(K)
            out["omega"][m] = collision_strengths(T, P, target, n_target,
                                                  float(sym["g"]))
        if "R" in keep:
            out["R"].append(R_all[m])
        if "K" in keep:
            out["K"].append((K, P))
        if "T" in keep:
            out["T"].append((T, P))
    return out
