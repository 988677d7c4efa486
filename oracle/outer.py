"""Outer-region propagation beyond r = a with long-range multipole coupling
(FP64 oracle).

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see the package docstring).

The paper matches at r = a and says nothing of the region beyond it; real
targets couple the channels there through the long-range multipole
potentials of the target, and production codes propagate the R-matrix
outwards before matching.  Read here as:

* for r >= a the channel functions obey u'' = (W(r) - E) u with
      W_ij(r) = [e_i + l_i (l_i + 1)/r^2 - 2z/r] delta_ij
                + sum_{lam = 1..lmax} beta^lam_ij / r^(lam + 1),
  beta^lam symmetric (Ry a0^(lam+1)), E and e_i in Ry;
* the reduced R-matrix Rr(r) = u(r) u'(r)^-1 (Rr(a) = a R(a)) is carried
  from a to A through n_sec sectors of equal width h; in a sector W is
  frozen at the sector's midpoint, W_s = U_s diag(eps) U_s^T, and with
  kappa^2 = E - eps, c = cos(kappa h), s = sin(kappa h)/kappa (cosh and
  sinh(|kappa| h)/|kappa| when kappa^2 < 0):
      Rr(r2) = U_s (c X + s)(c - kappa^2 s X)^-1 U_s^T,  X = U_s^T Rr(r1) U_s,
  which is exact for a constant W (the solutions of each decoupled channel
  are cos and sin);
* at A, R(A) = Rr(A)/A is matched to the Coulomb (open) and Whittaker
  (closed) functions at r = A by the same matching as at r = a; the
  multipole terms beyond A are dropped;
* or, with the asymptotic expansion switched on, the open-channel
  solutions at A are the coupled asymptotic series of Gailitis (J. Phys. B
  9 (1976) 843; Burke, "R-Matrix Theory of Atomic Collisions", 2011,
  Ch. 2), which keeps the multipole terms beyond A (see ``gailitis``); the
  closed channels keep their decaying Whittaker functions.  The paper is
  silent on all of this.
"""
import numpy as np
from scipy.special import loggamma

from .rmatrix import (r_matrix, channel_data, k_matrix, t_matrix,
                      collision_strengths)


def potential_matrix(r, e_thr, l, z, beta):
    """W(r) [n, n] for channel thresholds e_thr, angular momenta l, charge
    z and multipole coefficients beta [lmax, n, n] (lam = 1..lmax)."""
    e_thr = np.asarray(e_thr, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    W = np.diag(e_thr + l * (l + 1.0) / r ** 2 - 2.0 * z / r)
    beta = np.asarray(beta, dtype=np.float64)
    for lam in range(beta.shape[0]):
        W = W + beta[lam] / r ** (lam + 2)
    return W


def sectors(W_of_r, a, A, n_sec):
    """[(h, eps, U)] of the n_sec equal sectors of [a, A], W frozen at each
    sector's midpoint."""
    out = []
    if n_sec < 1 or A <= a:
        return out
    h = (A - a) / n_sec
    for s in range(n_sec):
        Wm = W_of_r(a + (s + 0.5) * h)
        eps, U = np.linalg.eigh(0.5 * (Wm + Wm.T))
        out.append((h, eps, U))
    return out


def _cs(k2, h):
    """c = cos(kappa h), s = sin(kappa h)/kappa for kappa^2 = k2 (either sign)."""
    c = np.empty_like(k2)
    s = np.empty_like(k2)
    op = k2 > 0
    k = np.sqrt(np.abs(k2))
    c[op] = np.cos(k[op] * h)
    s[op] = np.sin(k[op] * h) / k[op]
    cl = k2 < 0
    c[cl] = np.cosh(k[cl] * h)
    s[cl] = np.sinh(k[cl] * h) / k[cl]
    z = k2 == 0
    c[z] = 1.0
    s[z] = h
    return c, s


def propagate(Rr, secs, E):
    """Carry Rr = u u'^-1 through the sectors at energy E."""
    Rr = np.asarray(Rr, dtype=np.float64)
    for h, eps, U in secs:
        X = U.T @ Rr @ U
        k2 = E - eps
        c, s = _cs(k2, h)
        N = c[:, None] * X + np.diag(s)
        D = np.diag(c) - (k2 * s)[:, None] * X
        Y = N @ np.linalg.inv(D)
        Rr = U @ (0.5 * (Y + Y.T)) @ U.T
    return Rr


def outer_sectors(sym, prop):
    """Sectors of a symmetry dict for prop = {"A", "n_sec", "beta"} (beta in
    the symmetry's channel order)."""
    def Wr(r):
        return potential_matrix(r, sym["e_thr"], sym["l"], sym["z"],
                                prop["beta"])
    return sectors(Wr, sym["a"], prop["A"], prop["n_sec"])


def r_matrix_at_A(sym, prop, E, secs=None):
    """R(A) at one energy: the pole sum at r = a, propagated to A."""
    secs = outer_sectors(sym, prop) if secs is None else secs
    a = sym["a"]
    Ra = r_matrix(sym["E_pole"], sym["w"], a, E)[0]
    return propagate(a * Ra, secs, E) / prop["A"]


def k_matrix_propagated(sym, prop, E):
    """(K, P) at one energy with matching at r = A."""
    RA = r_matrix_at_A(sym, prop, E)
    A = prop["A"]
    cd = channel_data(np.array([E]), sym["e_thr"], sym["l"], sym["z"], A)
    cd1 = {k: v[0] for k, v in cd.items()}
    return k_matrix(RA, A, cd1["open"], cd1["s"], cd1["c"], cd1["sp"],
                    cd1["cp"], cd1["L"])


def sweep_propagated(sym, prop, E, n_target=None):
    """Omega [m, P] over a mesh with the outer propagation (with the
    asymptotic expansion when prop has "gailitis_terms" > 0)."""
    if prop.get("gailitis_terms", 0) > 0:
        return sweep_propagated_gailitis(sym, prop, E, n_target)[0]
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    n = sym["w"].shape[0]
    target = sym.get("target")
    target = np.arange(n) if target is None else np.asarray(target)
    if n_target is None:
        n_target = int(target.max()) + 1
    P = n_target * (n_target + 1) // 2
    secs = outer_sectors(sym, prop)
    A = prop["A"]
    cd = channel_data(E, sym["e_thr"], sym["l"], sym["z"], A)
    out = np.zeros((E.size, P))
    for m, Ee in enumerate(E):
        a = sym["a"]
        Ra = r_matrix(sym["E_pole"], sym["w"], a, Ee)[0]
        RA = propagate(a * Ra, secs, Ee) / A
        c1 = {k: v[m] for k, v in cd.items()}
        K, Pk = k_matrix(RA, A, c1["open"], c1["s"], c1["c"], c1["sp"],
                         c1["cp"], c1["L"])
        if Pk.size == 0:
            continue
        out[m] = collision_strengths(t_matrix(K), Pk, target, n_target,
                                     sym.get("g", 1.0))
    return out


# ---------------------------------------------------------------------------
# Asymptotic expansion beyond A.
#
# For r >= A the equations u'' = (W(r) - E) u keep their multipole terms.
# A solution that behaves as exp(i theta_j) in open channel j is written
#     u_i(r) = g_ij(r) exp(i theta_j(r)),  g_ij(r) = sum_p c^p_ij r^-p,
#     theta_j = k_j r - eta_j ln(2 k_j r) - l_j pi/2 + sigma_j,
# with k_j^2 = E - e_j, eta_j = -z/k_j and sigma_j = arg Gamma(l_j + 1 +
# i eta_j).  Putting this into the equations and collecting the powers of
# 1/r gives, with br_i(p) = (p + i eta_j - l_i - 1)(p + i eta_j + l_i) and
# V^p_i = sum_lam sum_m beta^lam_im c^(p - lam)_m,
#     (k_i^2 - k_j^2) c^(p+1)_i = 2 i k_j p c^p_i - br_i(p) c^(p-1)_i + V^p_i
# for every p >= 0.  Where k_i = k_j (e_i = e_j, channel j itself among
# them) the left side vanishes and the same relation, taken at p + 1 and
# solved for c^p_i, gives c^p_i = (br_i(p) c^(p-1)_i - V^p_i)/(2 i k_j p).
# c^0_ij = delta_ij, c^p = 0 for p < 0.  Without coupling the series is the
# asymptotic series of the Coulomb function H+ = G + iF (DLMF 33.11.1).
# The series is asymptotic: it is summed up to its smallest term.
# ---------------------------------------------------------------------------

GAILITIS_CONV = 1e-16   # a term this small (relative to g ~ 1) ends the sum
GAILITIS_FLAG = 1e-6    # a first omitted term above this flags the channel


def coulomb_phase(l, eta):
    """sigma_l(eta) = arg Gamma(l + 1 + i eta), the Coulomb phase shift."""
    return np.asarray(loggamma(np.asarray(l, dtype=np.float64) + 1.0
                               + 1j * np.asarray(eta, dtype=np.float64)).imag)


def gailitis_column(j, E, e_thr, l, z, beta, r, max_terms):
    """(g [n], g' [n], nonconv) of the solution that starts as exp(i theta_j)
    in open channel j, summed at radius r.  A term is added while its size
    T_p = max_i |c^p_i| r^-p does not exceed the last one's (T_0 = 1): the
    first term that grows ends the sum unadded (the smallest-term
    truncation of an asymptotic series); a term below GAILITIS_CONV ends it
    after being added.  nonconv: the first omitted term (or, at max_terms,
    the last added one) exceeds GAILITIS_FLAG."""
    e_thr = np.asarray(e_thr, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    n = e_thr.size
    k2 = E - e_thr
    kj = np.sqrt(k2[j])
    eta = -float(z) / kj
    deg = e_thr == e_thr[j]

    def br(p):
        return (p + 1j * eta - l - 1.0) * (p + 1j * eta + l)

    c = {0: np.zeros(n, dtype=complex)}
    c[0][j] = 1.0

    def cget(p):
        return c[p] if p >= 0 else np.zeros(n, dtype=complex)

    def V(p):
        v = np.zeros(n, dtype=complex)
        for lam in range(1, beta.shape[0] + 1):
            v = v + beta[lam - 1] @ cget(p - lam)
        return v

    g = c[0].copy()
    gp = np.zeros(n, dtype=complex)
    t_prev = 1.0
    nonconv = False
    for p in range(1, max_terms + 1):
        cp = np.empty(n, dtype=complex)
        Vp = V(p)
        cp[deg] = (br(p)[deg] * cget(p - 1)[deg] - Vp[deg]) / (2j * kj * p)
        Vq = V(p - 1)
        nd = ~deg
        cp[nd] = ((2j * kj * (p - 1)) * cget(p - 1)[nd]
                  - br(p - 1)[nd] * cget(p - 2)[nd] + Vq[nd]) / (k2[nd] - k2[j])
        c[p] = cp
        t = float(np.max(np.abs(cp))) * r ** (-p)
        if t > t_prev:
            nonconv = t > GAILITIS_FLAG
            return g, gp, nonconv
        g = g + cp * r ** (-p)
        gp = gp - p * cp * r ** (-p - 1)
        if t <= GAILITIS_CONV:
            return g, gp, False
        t_prev = t
    nonconv = t_prev > GAILITIS_FLAG
    return g, gp, nonconv


def gailitis(E, e_thr, l, z, beta, r, max_terms=40):
    """Asymptotic solutions at radius r, one per open channel j (ascending
    channel index), normalised like s = k^-1/2 F and c = k^-1/2 G:
        S_ij = k_j^-1/2 Im(g_ij e^{i theta_j}),  C_ij = k_j^-1/2 Re(...),
    and their r-derivatives Sp, Cp (u' = (g' + i theta_j' g) e^{i theta_j},
    theta_j' = k_j - eta_j / r).  Returns (S, C, Sp, Cp [n, n_o], P,
    nonconv [n_o])."""
    e_thr = np.asarray(e_thr, dtype=np.float64)
    l = np.asarray(l, dtype=np.float64)
    P = np.nonzero(E > e_thr)[0]
    n = e_thr.size
    S = np.zeros((n, P.size))
    C = np.zeros((n, P.size))
    Sp = np.zeros((n, P.size))
    Cp = np.zeros((n, P.size))
    flags = np.zeros(P.size, dtype=bool)
    for col, j in enumerate(P):
        kj = np.sqrt(E - e_thr[j])
        eta = -float(z) / kj
        theta = (kj * r - eta * np.log(2.0 * kj * r) - l[j] * np.pi / 2.0
                 + coulomb_phase(l[j], eta))
        g, gp, flags[col] = gailitis_column(j, E, e_thr, l, z, beta, r,
                                            max_terms)
        ph = np.exp(1j * theta) / np.sqrt(kj)
        u = g * ph
        up = (gp + 1j * (kj - eta / r) * g) * ph
        S[:, col], C[:, col] = u.imag, u.real
        Sp[:, col], Cp[:, col] = up.imag, up.real
    return S, C, Sp, Cp, P, flags


def k_matrix_asymptotic(R, r, S, C, Sp, Cp, P, L):
    """Open-open K-matrix from u(r) = R r u'(r) with coupled open-channel
    solutions: every open column j is S_j + sum_i C_i K_ij plus the closed
    channels' decaying functions (e, r e') = (1, L)/sqrt(1 + L^2) with
    coefficients X, so
        [C - R r Cp | diag(e_Q) - R diag(r e'_Q)] [K; X] = R r Sp - S
    with the columns of C in the places of the open channels.  L [n] holds
    the closed channels' r W'/W (ignored elsewhere).  Returns K [n_o, n_o]."""
    n = R.shape[0]
    if P.size == 0:
        return np.zeros((0, 0))
    A = np.zeros((n, n))
    closed = np.setdiff1d(np.arange(n), P)
    A[:, P] = C - r * (R @ Cp)
    if closed.size:
        L = np.asarray(L, dtype=np.float64)
        nrm = np.hypot(1.0, L[closed])
        A[closed, closed] += 1.0 / nrm
        A[:, closed] -= R[:, closed] * (L[closed] / nrm)[None, :]
    B = r * (R @ Sp) - S
    Z = np.linalg.solve(A, B)
    return Z[P, :]


def k_matrix_propagated_gailitis(sym, prop, E):
    """(K, P, nonconv) at one energy: propagation to A, matching to the
    asymptotic expansion with prop["gailitis_terms"] terms at most (K
    symmetrised, as the sweep uses it)."""
    A = prop["A"]
    RA = r_matrix_at_A(sym, prop, E)
    S, C, Sp, Cp, P, nc = gailitis(E, sym["e_thr"], sym["l"], sym["z"],
                                   np.asarray(prop["beta"], dtype=np.float64),
                                   A, prop["gailitis_terms"])
    if P.size == 0:
        return np.zeros((0, 0)), P, False
    cd = channel_data(np.array([E]), sym["e_thr"], sym["l"], sym["z"], A)
    K = k_matrix_asymptotic(RA, A, S, C, Sp, Cp, P, cd["L"][0])
    return 0.5 * (K + K.T), P, bool(nc.any())


def sweep_propagated_gailitis(sym, prop, E, n_target=None):
    """(Omega [m, P], nonconv [m] bool) over a mesh: propagation to A, then
    matching to the asymptotic expansion with prop["gailitis_terms"] terms
    at most."""
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    n = sym["w"].shape[0]
    target = sym.get("target")
    target = np.arange(n) if target is None else np.asarray(target)
    if n_target is None:
        n_target = int(target.max()) + 1
    Pn = n_target * (n_target + 1) // 2
    secs = outer_sectors(sym, prop)
    A = prop["A"]
    beta = np.asarray(prop["beta"], dtype=np.float64)
    cd = channel_data(E, sym["e_thr"], sym["l"], sym["z"], A)
    out = np.zeros((E.size, Pn))
    flags = np.zeros(E.size, dtype=bool)
    for m, Ee in enumerate(E):
        Ra = r_matrix(sym["E_pole"], sym["w"], sym["a"], Ee)[0]
        RA = propagate(sym["a"] * Ra, secs, Ee) / A
        S, C, Sp, Cp, P, nc = gailitis(Ee, sym["e_thr"], sym["l"], sym["z"],
                                       beta, A, prop["gailitis_terms"])
        if P.size == 0:
            continue
        flags[m] = bool(nc.any())
        K = k_matrix_asymptotic(RA, A, S, C, Sp, Cp, P, cd["L"][m])
        out[m] = collision_strengths(t_matrix(0.5 * (K + K.T)), P, target,
                                     n_target, sym.get("g", 1.0))
    return out, flags
