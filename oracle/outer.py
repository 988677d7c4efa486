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
  multipole terms beyond A are dropped.
"""
import numpy as np

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
    """Omega [m, P] over a mesh with the outer propagation."""
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
