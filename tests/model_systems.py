"""Model inner regions with known answers, for pinning the oracle.

A short-range model potential plus the Coulomb tail defines, on [0, a], the
radial problem (Rydberg units)

    u_i'' = sum_j [ (l_i(l_i+1)/r^2 - 2z/r + e_i - E) delta_ij + U_ij(r) ] u_j

Two independent routes give its boundary quantities:

* ``bloch_poles``: the Bloch-augmented Hamiltonian (Bloch constant b = 0) in a
  polynomial basis r P_m(2r/a - 1) per channel; its eigenvalues are the poles
  E_k and sqrt(2) times the eigenvector's surface value is w_ik (the inputs
  the outer-region sweep receives from the inner region);
* ``ode_rmatrix`` / ``ode_kmatrix``: direct integration of the coupled
  equations (scipy DOP853), giving R = u(a) [a u'(a)]^-1 and, continued past
  r = a, the K-matrix fitted to mpmath's Coulomb functions.

Nothing here imports the oracle or the HIP path.
"""
import math

import mpmath
import numpy as np
import scipy.integrate
import scipy.linalg
from numpy.polynomial import legendre as npleg


def gaussian_potential(depth, r0):
    return lambda r: -depth * np.exp(-(r / r0) ** 2)


class ModelSystem:
    """n-channel model: thresholds e, angular momenta l, charge z, radius a,
    and U(r) -> [n, n] symmetric short-range potential matrix."""

    def __init__(self, e, l, z, a, U):
        self.e = np.asarray(e, dtype=np.float64)
        self.l = np.asarray(l, dtype=np.int64)
        self.z = float(z)
        self.a = float(a)
        self.U = U
        self.n = self.e.size

    def coupling(self, r):
        n = self.n
        W = np.array(self.U(r), dtype=np.float64).reshape(n, n)
        W = W + np.diag(self.l * (self.l + 1) / r ** 2 - 2.0 * self.z / r
                        + self.e)
        return W


def bloch_poles(sys, N=80, Q=None):
    """Poles E_k [n*N] and amplitudes w [n, n*N] from the Bloch eigenproblem."""
    a, n = sys.a, sys.n
    Q = Q or N + 80
    xg, wg = npleg.leggauss(Q)
    r = 0.5 * a * (xg + 1.0)
    wr = 0.5 * a * wg
    V = npleg.legvander(xg, N - 1)                       # P_m(x) [Q, N]
    dV = np.stack([npleg.legval(xg, npleg.legder(np.eye(N)[m]))
                   for m in range(N)], axis=1)          # P_m'(x)
    phi = r[:, None] * V
    dphi = V + r[:, None] * (2.0 / a) * dV
    T = (dphi * wr[:, None]).T @ dphi
    O1 = (phi * wr[:, None]).T @ phi
    H = np.zeros((n * N, n * N))
    O = np.zeros((n * N, n * N))
    Ur = np.stack([np.array(sys.U(ri), dtype=np.float64).reshape(n, n)
                   for ri in r])                          # [Q, n, n]
    for i in range(n):
        diag = (sys.l[i] * (sys.l[i] + 1) / r ** 2 - 2.0 * sys.z / r
                + sys.e[i])
        for j in range(n):
            pot = Ur[:, i, j] + (diag if i == j else 0.0)
            blk = (phi * (wr * pot)[:, None]).T @ phi
            if i == j:
                blk = blk + T
                O[i * N:(i + 1) * N, i * N:(i + 1) * N] = O1
            H[i * N:(i + 1) * N, j * N:(j + 1) * N] = blk
    H = 0.5 * (H + H.T)
    Ek, C = scipy.linalg.eigh(H, O)
    surf = a * np.ones(N)                                 # phi_m(a) = a P_m(1)
    w = np.stack([math.sqrt(2.0) * (surf @ C[i * N:(i + 1) * N, :])
                  for i in range(n)])
    return Ek, w


def _regular_start(sys, E, r0):
    """Regular solutions near r = 0: column j ~ r^(l_j+1) (1 - z r/(l_j+1))."""
    n = sys.n
    u = np.zeros((n, n))
    up = np.zeros((n, n))
    for j in range(n):
        L = sys.l[j]
        c1 = -sys.z / (L + 1.0)
        u[j, j] = r0 ** (L + 1) * (1.0 + c1 * r0)
        up[j, j] = (L + 1) * r0 ** L + (L + 2) * c1 * r0 ** (L + 1)
    return u, up


def _integrate(sys, E, r_from, r_to, u, up, rtol=1e-13):
    n = sys.n

    def rhs(r, y):
        Y = y.reshape(2, n, n)
        W = sys.coupling(r) - E * np.eye(n)
        return np.concatenate([Y[1].ravel(), (W @ Y[0]).ravel()])

    y0 = np.concatenate([u.ravel(), up.ravel()])
    sol = scipy.integrate.solve_ivp(rhs, (r_from, r_to), y0, method="DOP853",
                                    rtol=rtol, atol=1e-300)
    Y = sol.y[:, -1].reshape(2, n, n)
    return Y[0], Y[1]


def ode_rmatrix(sys, E, r0=1e-5):
    """R(E) = u(a) [a u'(a)]^-1 from regular solutions integrated to r = a."""
    u, up = _regular_start(sys, E, r0)
    ua, upa = _integrate(sys, E, r0, sys.a, u, up)
    return ua @ np.linalg.inv(sys.a * upa)


def _coulomb_mp(l, z, k, r):
    """s, c, s', c' at radius r from mpmath (independent of the oracle)."""
    with mpmath.workdps(30):
        kk = mpmath.mpf(k)
        eta = -z / kk
        rho = kk * r
        F = mpmath.coulombf(l, eta, rho)
        G = mpmath.coulombg(l, eta, rho)
        Fp = mpmath.diff(lambda x: mpmath.coulombf(l, eta, x), rho)
        Gp = mpmath.diff(lambda x: mpmath.coulombg(l, eta, x), rho)
        sk = mpmath.sqrt(kk)
        return (float(F / sk), float(G / sk), float(Fp * sk), float(Gp * sk))


def ode_kmatrix(sys, E, r_out, r0=1e-5):
    """K-matrix of the open channels from integration out to r_out > a.

    Closed channels must have decayed by r_out: the physical solutions are
    the combinations whose closed components vanish there.  Open components
    are then fitted to s A + c B (Wronskian c s' - s c' = 1) and K = B A^-1.
    """
    u, up = _regular_start(sys, E, r0)
    U, Up = _integrate(sys, E, r0, r_out, u, up)
    P = np.nonzero(E > sys.e)[0]
    Qc = np.nonzero(E <= sys.e)[0]
    if Qc.size:
        # null space of the closed rows (value and derivative) at r_out
        M = np.vstack([U[Qc], Up[Qc]])
        _, sv, vt = np.linalg.svd(M)
        basis = vt[Qc.size:].T            # n x n_o
        U = U @ basis
        Up = Up @ basis
    A = np.zeros((P.size, U.shape[1]))
    B = np.zeros((P.size, U.shape[1]))
    for row, i in enumerate(P):
        s, c, sp, cp = _coulomb_mp(int(sys.l[i]), sys.z,
                                   math.sqrt(E - sys.e[i]), r_out)
        A[row] = c * Up[i] - cp * U[i]
        B[row] = sp * U[i] - s * Up[i]
    return B @ np.linalg.inv(A)


def square_well_poles(V0, a, n_poles):
    """Analytic Bloch poles of -u'' - V0 u on [0, a] with u'(a) = 0 (b = 0):
    K_m a = (m + 1/2) pi, E_m = K_m^2 - V0, u_m(a)^2 = 2/a so w_m^2 = 4/a."""
    m = np.arange(n_poles)
    Km = (m + 0.5) * math.pi / a
    return Km ** 2 - V0, np.full((1, n_poles), 2.0 / math.sqrt(a))


def square_well_tail(V0, a, E, n_poles):
    """sum_{m >= n_poles} 2/((m+1/2)^2 pi^2 - x^2), x = sqrt(E + V0) a.

    By partial fractions with y = x/pi the sum telescopes into digammas:
    (psi(n + 1/2 + y) - psi(n + 1/2 - y)) / (pi^2 y).
    """
    with mpmath.workdps(40):
        y = mpmath.sqrt(mpmath.mpf(E) + V0) * a / mpmath.pi
        h = mpmath.mpf(n_poles) + mpmath.mpf(1) / 2
        return float((mpmath.digamma(h + y) - mpmath.digamma(h - y))
                     / (mpmath.pi ** 2 * y))
