"""Photoionization cross sections from the outer-region solve (FP64 oracle).

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see the package docstring).

The paper's photoionization runs (Sec. 2 and 3: the dipole-pair stage and
the outer-region module for photoionization, Tables 1-2; Sec. 4-5: the
nitrogen, oxygen, krypton, xenon and W3+ cross sections) reuse the
scattering solve at every energy and add the bound-free dipole matrix
elements between the initial state and the inner-region states of each
dipole-allowed final symmetry.  The paper writes no formula for this step;
it is standard R-matrix theory (Burke, "R-Matrix Theory of Atomic
Collisions", 2011, the photoionization chapter), read here without
radiation damping:

* A solution of energy E inside r < a is sum_k A_k psi_k with
  A_k = sum_i (w_ik / sqrt2) u_i'(a) / (E_k - E): the Bloch relation with
  b = 0 in the convention R_ij = (1/2a) sum_k w_ik w_jk / (E_k - E), i.e.
  w = sqrt2 u_k(a) (the same reading as the scattering path).
* For the real K-matrix solution j, u_ij'(a) = s_i' delta_ij + c_i' K_ij on
  an open channel i and e_i' X_ij on a closed one, [K; X] the solution of
  the matching system.  Its dipole amplitude with the initial state is
      M_j = sum_k A_jk d_k = sum_i u_ij'(a) g_i,
      g_i = (1/sqrt2) sum_k w_ik d_k / (E_k - E),
  d_k the dipole matrix element between inner-region state k and the
  initial state (angular factors included in d).
* s = k^-1/2 F and c = k^-1/2 G are normalised to pi delta(E - E') (E in
  Ry), so the energy-normalised incoming-wave solutions are
  pi^-1/2 Psi^K (1 - iK)^-1; summed over the final channels the squared
  amplitudes give the dipole strength
      S(E) = (1/pi) M (1 + K^2)^-1 M^T.
* sigma(E) = (4 pi^2 alpha a0^2 / 3) omega S(E) with the photon energy
  omega = E - e0 in Ry (e0 the initial-state energy on the same scale as
  the thresholds), in Mb; summed over the final symmetries.
"""
import numpy as np

from .rmatrix import r_matrix, channel_data

ALPHA = 7.2973525693e-3          # fine-structure constant
A0_SQ_MB = 28.00285205           # a0^2 in Mb
SIGMA_CONST = 4.0 * np.pi ** 2 * ALPHA * A0_SQ_MB / 3.0   # Mb per (Ry a0^2/Ry)


def dipole_pole_sum(E_pole, w, d, E):
    """g_i(E) = (1/sqrt2) sum_k w_ik d_k / (E_k - E)."""
    w = np.asarray(w, dtype=np.float64)
    dk = np.asarray(d, dtype=np.float64) / (np.asarray(E_pole) - E)
    return (w @ dk) / np.sqrt(2.0)


def matching_solution(R, a, cd):
    """Full solution [K; X] (n x n_open, channels in their own order) of
        (D1 - R D2) Z = R[:, P] diag(a s'_P) - [diag(s_P); 0],
    D1 = diag(c_P, e_Q), D2 = diag(a c'_P, a e'_Q), (e, a e') the closed
    channel function at r = a scaled to unit length; also returns P and the
    diagonal of D2."""
    op = cd["open"]
    P = np.nonzero(op)[0]
    n = R.shape[0]
    d1 = np.empty(n)
    d2 = np.empty(n)
    d1[op] = cd["c"][op]
    d2[op] = a * cd["cp"][op]
    L = cd["L"][~op]
    nrm = np.hypot(1.0, L)
    d1[~op] = 1.0 / nrm
    d2[~op] = L / nrm
    if P.size == 0:
        return np.zeros((n, 0)), P, d2
    A = np.diag(d1) - R * d2[None, :]
    B = R[:, P] * (a * cd["sp"][P])[None, :]
    B[P, np.arange(P.size)] -= cd["s"][P]
    return np.linalg.solve(A, B), P, d2


def dipole_strength(R, g, a, cd):
    """S(E) from R, the dipole pole sum g and the channel data at E."""
    Z, P, d2 = matching_solution(R, a, cd)
    if P.size == 0:
        return 0.0
    M = (a * cd["sp"][P] * g[P] + Z.T @ (d2 * g)) / a
    K = Z[P, :]
    K = 0.5 * (K + K.T)
    return float(M @ np.linalg.solve(np.eye(P.size) + K @ K, M)) / np.pi


def photoionization(syms, dips, E, e0):
    """sigma(E) in Mb, summed over the final symmetries `syms` (dicts as for
    rmatrix.sweep) with dipole vectors `dips` (one [N_H] array each)."""
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    out = np.zeros(E.size)
    for sym, d in zip(syms, dips):
        cd = channel_data(E, sym["e_thr"], sym["l"], sym["z"], sym["a"])
        for m, Ee in enumerate(E):
            R = r_matrix(sym["E_pole"], sym["w"], sym["a"], Ee)[0]
            cd1 = {k: v[m] for k, v in cd.items()}
            g = dipole_pole_sum(sym["E_pole"], sym["w"], d, Ee)
            out[m] += dipole_strength(R, g, sym["a"], cd1)
    return SIGMA_CONST * (E - e0) * out


# ---------------------------------------------------------------------------
# Radiation damping.
#
# The paper's photoionization module damps its resonances (Sec. 3: the
# damped outer-region module of Tables 1-2) and prints no formula.  Read as
# the optical-potential damping of standard R-matrix theory: each
# inner-region state k decays radiatively with width Gamma_k, so the
# effective Hamiltonian is H - i sum_k (Gamma_k / 2) |psi_k><psi_k| and its
# inner-region eigenvalues are E_k - i Gamma_k / 2.  The photoionization
# cross section is then the flux into the open channels of the driven
# solution (E - H_eff) psi = D Psi_0 with purely outgoing waves outside:
#   inside r < a   psi = sum_k A_k psi_k,
#                  A_k = [sum_i (w_ik / sqrt2) u_i'(a) - d_k] / (E_k - i Gamma_k/2 - E),
#   hence          u(a) = a R_c u'(a) - g_c   with R_c, g_c the pole sums of
#                  the damped pole energies;
#   outside        u_i = O_i alpha_i (open, O = c + i s, outgoing) and
#                  e_i beta_i (closed, decaying),
# so (diag(d1) - R_c diag(d2)) x = -g_c for x = [alpha; beta], with
# d1 = c + i s, d2 = a (c' + i s') on open channels and (e, a e') on closed
# ones.  The flux through r = a in open channel f is |alpha_f|^2 (c s' -
# s c' = 1), and with Gamma = 0 the same solution gives alpha_P =
# -(1 - iK)^-1 M, so sum_f |alpha_f|^2 = pi S(E): the damped strength is
#   S_damp(E) = (1/pi) sum_{f open} |alpha_f|^2,
# equal to the undamped S(E) when every width vanishes.  The widths are an
# input per pole (the radiative widths of the inner-region states).
# ---------------------------------------------------------------------------

def damped_pole_sums(E_pole, w, d, widths, a, E):
    """Complex R_c [n, n] and g_c [n] with pole energies E_k - i Gamma_k/2."""
    w = np.asarray(w, dtype=np.float64)
    dk = 1.0 / (np.asarray(E_pole, dtype=np.float64)
                - 0.5j * np.asarray(widths, dtype=np.float64) - E)
    R = ((w * dk[None, :]) @ w.T) / (2.0 * a)
    g = (w @ (np.asarray(d, dtype=np.float64) * dk)) / np.sqrt(2.0)
    return R, g


def outgoing_channel_values(a, cd):
    """d1 = u(a) and d2 = a u'(a) per unit amplitude of the outgoing-wave
    channel functions: c + i s and a (c' + i s') on open channels, the
    closed function (e, a e') scaled to unit length on closed ones."""
    op = cd["open"]
    n = op.size
    d1 = np.empty(n, dtype=np.complex128)
    d2 = np.empty(n, dtype=np.complex128)
    d1[op] = cd["c"][op] + 1j * cd["s"][op]
    d2[op] = a * (cd["cp"][op] + 1j * cd["sp"][op])
    L = cd["L"][~op]
    nrm = np.hypot(1.0, L)
    d1[~op] = 1.0 / nrm
    d2[~op] = L / nrm
    return d1, d2


def driven_solution(R, g, a, cd):
    """x = [alpha; beta] (channels in their own order) of
    (diag(d1) - R diag(d2)) x = -g, and the open-channel list P."""
    d1, d2 = outgoing_channel_values(a, cd)
    A = np.diag(d1) - R * d2[None, :]
    x = np.linalg.solve(A, -np.asarray(g, dtype=np.complex128))
    return x, np.nonzero(cd["open"])[0], d2


def damped_dipole_strength(R, g, a, cd):
    """S_damp(E) = (1/pi) sum over open channels of |alpha_f|^2."""
    x, P, _ = driven_solution(R, g, a, cd)
    return float(np.sum(np.abs(x[P]) ** 2)) / np.pi


def inner_amplitudes(E_pole, w, d, widths, a, x, d2, E):
    """A_k of the driven solution inside r < a, from u'(a) = d2 x / a."""
    up = d2 * x / a
    num = (np.asarray(w, dtype=np.float64).T @ up) / np.sqrt(2.0) \
        - np.asarray(d, dtype=np.float64)
    return num / (np.asarray(E_pole) - 0.5j * np.asarray(widths) - E)


def photoionization_damped(syms, dips, widths, E, e0):
    """sigma(E) in Mb with radiation damping: as photoionization(), with the
    widths Gamma_k (one [N_H] array per symmetry) on the pole energies."""
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    out = np.zeros(E.size)
    for sym, d, G in zip(syms, dips, widths):
        cd = channel_data(E, sym["e_thr"], sym["l"], sym["z"], sym["a"])
        for m, Ee in enumerate(E):
            cd1 = {k: v[m] for k, v in cd.items()}
            if not cd1["open"].any():
                continue
            R, g = damped_pole_sums(sym["E_pole"], sym["w"], d, G, sym["a"], Ee)
            out[m] += damped_dipole_strength(R, g, sym["a"], cd1)
    return SIGMA_CONST * (E - e0) * out
