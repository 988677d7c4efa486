"""Inner-region eigen-solve that produces the path's poles (FP64 oracle).

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see the package docstring).

The paper diagonalises the inner-region Hamiltonian of each symmetry in
full (Sec. 2-3: every eigenvalue and eigenvector, dimensions of 2K to 200K,
ScaLAPACK); the eigenvalues are the poles E_k of Eq. 1 and the eigenvectors'
surface values give the amplitudes w_ik.  The paper's Hamiltonians come from
atomic structure data that are not published; a multichannel model stands
in, read as:

* channels i with thresholds e_i, angular momenta l_i and residual charge z;
  on [0, a] the radial functions obey
      u_i'' = sum_j [(l_i (l_i + 1)/r^2 - 2z/r + e_i - E) delta_ij + U_ij(r)] u_j,
      U_ij(r) = -depth_ij exp(-(r / range_ij)^2)   (symmetric);
* basis per channel: phi_m(r) = sqrt(2/a) sin(kappa_m r), kappa_m a =
  (m + 1/2) pi, m = 0..N-1 (u(0) = 0, u'(a) = 0, orthonormal), so the Bloch
  operator with b = 0 adds nothing and the kinetic part is diag(kappa_m^2);
* H_(i,m),(j,m') = kappa_m^2 delta_ij delta_mm'
                   + int_0^a phi_m W_ij phi_m' dr  (Gauss-Legendre, Q nodes),
  W_ij the potential matrix above without E;
* poles E_k: the eigenvalues of H (ascending); amplitudes
  w_ik = sqrt2 u_ik(a) = sqrt2 sum_m C_(i,m),k phi_m(a), phi_m(a) =
  sqrt(2/a) (-1)^m, in the convention R = (1/2a) sum_k w w / (E_k - E).
"""
import numpy as np


def quadrature(a, Q):
    """Gauss-Legendre nodes and weights on [0, a].

    The nodes are the zeros x = cos(theta) of the Legendre polynomial P_Q,
    found by Newton's method in theta (P_Q and P_{Q-1} from the three-term
    recurrence, dP_Q/dtheta = Q (x P_Q - P_{Q-1}) / sin(theta)) in extended
    precision, so that theta is exact to double rounding although the
    recurrence loses about Q ulps.  Mapping x to r = a (1 + x) / 2 would
    lose the relative accuracy of the nodes next to r = 0, where the
    centrifugal term l (l + 1) / r^2 makes the matrix elements sensitive to
    it; instead 1 - cos(theta) = 2 sin^2(theta/2) and 1 + cos(theta) =
    2 cos^2(theta/2), and the weight 2 / ((1 - x^2) P_Q'(x)^2) is
    formed with 1 - x^2 = sin^2(theta).
    """
    ld = np.longdouble
    pi = ld("3.14159265358979323846264338327950288")
    h = (Q + 1) // 2
    th = pi * (np.arange(h, dtype=ld) + ld(0.75)) / (ld(Q) + ld(0.5))

    def legendre(x):
        p0, p1 = np.ones_like(x), x.copy()
        for k in range(2, Q + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        return (x, np.ones_like(x)) if Q == 1 else (p1, p0)

    # quadratic convergence from guesses within a few per cent: the step
    # falls below 1e-17 theta by the fifth iteration; one more polishes
    polish = False
    for _ in range(12):
        pq, pm = legendre(np.cos(th))
        step = pq * np.sin(th) / (Q * (np.cos(th) * pq - pm))
        th = th - step
        if polish:
            break
        polish = bool(np.all(np.abs(step) <= ld(1e-17) * np.abs(th)))
    x = np.cos(th)
    pq, pm = legendre(x)
    # P_Q'(x) = Q (x P_Q - P_{Q-1}) / (x^2 - 1) with x^2 - 1 = -sin^2(theta)
    wt = 2 * np.sin(th) ** 2 / (Q * (x * pq - pm)) ** 2
    # x = -cos(theta) (r near 0) for the first half, +cos(theta) mirrored
    r_lo = a * np.sin(th / 2) ** 2             # a (1 - cos theta) / 2
    r_hi = a * np.cos(th / 2) ** 2
    r = np.concatenate([r_lo, r_hi[: Q - h][::-1]]).astype(np.float64)
    w = (a * np.concatenate([wt, wt[: Q - h][::-1]]) / 2).astype(np.float64)
    return r, w


def basis(a, N, r):
    """phi_m(r) [len(r), N] and kappa_m [N]."""
    kap = (np.arange(N) + 0.5) * np.pi / a
    return np.sqrt(2.0 / a) * np.sin(np.outer(r, kap)), kap


def potential(model, r):
    """W(r) [len(r), n, n] without E."""
    e = np.asarray(model["e_thr"], dtype=np.float64)
    l = np.asarray(model["l"], dtype=np.float64)
    D = np.asarray(model["depth"], dtype=np.float64)
    Rg = np.asarray(model["range"], dtype=np.float64)
    W = -D[None] * np.exp(-(r[:, None, None] / Rg[None]) ** 2)
    diag = l[None] * (l[None] + 1.0) / r[:, None] ** 2 - 2.0 * model["z"] / r[:, None] + e[None]
    n = e.size
    W[:, np.arange(n), np.arange(n)] += diag
    return W


def hamiltonian(model, N, Q):
    """H [n N, n N], channel-major ((i, m) -> i N + m)."""
    a = model["a"]
    r, wq = quadrature(a, Q)
    phi, kap = basis(a, N, r)
    W = potential(model, r)
    n = W.shape[1]
    H = np.zeros((n * N, n * N))
    for i in range(n):
        for j in range(n):
            H[i * N:(i + 1) * N, j * N:(j + 1) * N] = \
                (phi * (wq * W[:, i, j])[:, None]).T @ phi
    H[np.arange(n * N), np.arange(n * N)] += np.tile(kap ** 2, n)
    return 0.5 * (H + H.T)


def inner_region(model, N, Q=None):
    """(E_pole [n N] ascending, w [n, n N])."""
    Q = Q or N + 48
    H = hamiltonian(model, N, Q)
    E, C = np.linalg.eigh(H)
    a = model["a"]
    n = len(model["e_thr"])
    phia = np.sqrt(2.0 / a) * (-1.0) ** np.arange(N)
    w = np.sqrt(2.0) * np.einsum("imk,m->ik", C.reshape(n, N, -1), phia)
    return E, w
