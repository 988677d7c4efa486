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
from numpy.polynomial import legendre as npleg


def quadrature(a, Q):
    """Gauss-Legendre nodes and weights on [0, a]."""
    x, wq = npleg.leggauss(Q)
    return 0.5 * a * (x + 1.0), 0.5 * a * wq


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
