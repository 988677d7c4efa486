"""Post-processing of collision strengths on the energy mesh (FP64 oracle).

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see the package docstring).

The paper compares its cross sections with experiment after convolving them
with a Gaussian of stated full width at half maximum (Sec. 4, the nitrogen
and oxygen photoionization figures, 60 and 124 meV; Sec. 5, the krypton,
xenon and W3+ figures, 100 meV with statistical averaging over levels).  The
same operation applies to any function on the mesh; here it acts on
Omega(E).  The Maxwellian-averaged effective collision strength is the
standard quantity computed from Omega(E) downstream of such a sweep; the
paper does not state it.  Readings (both are definitions, written out
plainly here):

* Gaussian convolution on an ascending, possibly non-uniform mesh E_j:
      Omega~(E_i) = sum_j g_ij Omega(E_j) / sum_j g_ij,
      g_ij = exp(-(E_i - E_j)^2 / (2 s^2)) dE_j,   s = FWHM / (2 sqrt(2 ln 2)),
  with trapezoid weights dE_j (half intervals at the two ends) and the sum
  restricted to |E_i - E_j| <= 8 s.  Dividing by the discrete kernel sum
  keeps a constant unchanged, also at the ends of the mesh.
* Effective collision strength of the level pair (t, u) at temperature kT
  (Ry), with e = max(e_t, e_u) the upper level and eps = E - e the energy of
  the outgoing electron:
      Upsilon(kT) = int_0^inf Omega(eps) exp(-eps/kT) d(eps/kT),
  evaluated on the mesh points with E > e: Omega is held constant from the
  threshold to the first such point, the product Omega(eps) exp(-eps/kT) is
  integrated by the trapezoid rule between mesh points, and the integral is
  truncated at the last mesh point.
* Statistical averaging over the levels of a group (the fine-structure
  levels of a term, Sec. 5's averaged cross sections): cross sections
  averaged over initial levels with weights g_t and summed over final levels
  correspond to collision strengths summed over level pairs,
      Omega_G(a, b) = sum over unordered level pairs {t, u} with
                      {group(t), group(u)} = {a, b} of Omega(t, u),
  so that sigma(a -> b) = pi Omega_G(a, b) / (g_a k^2) with g_a = sum of g_t
  over the levels of a.  Each unordered level pair, elastic ones included,
  lands in exactly one unordered group pair.
* A one-point mesh has no trapezoid weight; its convolution is the identity
  (the limit of the normalised sum as the weight goes to zero).
"""
import numpy as np

CUTOFF_SIGMAS = 8.0
FWHM_PER_SIGMA = 2.0 * np.sqrt(2.0 * np.log(2.0))


def trapezoid_weights(E):
    """dE_j: half the span of the two intervals next to mesh point j."""
    E = np.asarray(E, dtype=np.float64)
    w = np.zeros_like(E)
    if E.size > 1:
        d = np.diff(E)
        w[:-1] += 0.5 * d
        w[1:] += 0.5 * d
    return w


def gaussian_convolve(E, omega, fwhm):
    """Omega~ on the same mesh; omega is [M, P] (energy-major)."""
    E = np.asarray(E, dtype=np.float64)
    om = np.asarray(omega, dtype=np.float64)
    s = fwhm / FWHM_PER_SIGMA
    dE = trapezoid_weights(E)
    out = np.empty_like(om)
    if E.size == 1:
        out[:] = om
        return out
    for i in range(E.size):
        lo = np.searchsorted(E, E[i] - CUTOFF_SIGMAS * s, side="left")
        hi = np.searchsorted(E, E[i] + CUTOFF_SIGMAS * s, side="right")
        x = E[lo:hi] - E[i]
        g = np.exp(-0.5 * (x / s) ** 2) * dE[lo:hi]
        out[i] = g @ om[lo:hi] / g.sum()
    return out


def effective_collision_strengths(E, omega, e_level, n_target, kT):
    """Upsilon [P, len(kT)] for the packed upper-triangle level pairs of
    omega [M, P] (P = n_target (n_target + 1) / 2)."""
    E = np.asarray(E, dtype=np.float64)
    om = np.asarray(omega, dtype=np.float64)
    e_level = np.asarray(e_level, dtype=np.float64)
    kT = np.atleast_1d(np.asarray(kT, dtype=np.float64))
    P = n_target * (n_target + 1) // 2
    ups = np.zeros((P, kT.size))
    for t in range(n_target):
        for u in range(t, n_target):
            p = t * n_target - t * (t - 1) // 2 + (u - t)
            e = max(e_level[t], e_level[u])
            i0 = np.searchsorted(E, e, side="right")  # first point above e
            if i0 >= E.size:
                continue
            eps = E[i0:] - e
            f = om[i0:, p]
            for q, T in enumerate(kT):
                x = eps / T
                y = f * np.exp(-x)
                total = f[0] * (1.0 - np.exp(-x[0]))    # threshold segment
                if x.size > 1:
                    total += np.sum(0.5 * (y[1:] + y[:-1]) * np.diff(x))
                ups[p, q] = total
    return ups


def group_collision_strengths(omega, n_target, group, n_group):
    """Omega_G [M, n_group (n_group + 1) / 2] from Omega [M, P] and the group
    index of every level (0 <= group[t] < n_group)."""
    om = np.asarray(omega, dtype=np.float64)
    group = np.asarray(group)
    Pg = n_group * (n_group + 1) // 2
    out = np.zeros((om.shape[0], Pg))
    for t in range(n_target):
        for u in range(t, n_target):
            p = t * n_target - t * (t - 1) // 2 + (u - t)
            a, b = sorted((int(group[t]), int(group[u])))
            q = a * n_group - a * (a - 1) // 2 + (b - a)
            out[:, q] += om[:, p]
    return out
