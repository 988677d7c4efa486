"""Asymptotic channel functions at the R-matrix boundary r = a (oracle).

TEST INFRASTRUCTURE: only tests/, smoke() and bench.py's cpu_baseline may use it.

The paper (Sec. 6) states only the R-matrix formation; the matching it feeds
needs, for every channel i at energy E (Rydberg units, radial equation
u'' + [k^2 - l(l+1)/r^2 + 2z/r] u = 0 outside r = a):

* open channel (E > e_i), k = sqrt(E - e_i), eta = -z/k, rho = k r:
  the regular and irregular Coulomb functions F_l(eta, rho), G_l(eta, rho)
  and their rho-derivatives, normalised by the Wronskian F'G - FG' = 1
  (Abramowitz & Stegun 14.1; DLMF 33.2).
* closed channel (E <= e_i), phi = sqrt(e_i - E), kappa = z/phi:
  the logarithmic derivative a W'(a)/W(a) of the decaying Whittaker function
  W_{kappa, l+1/2}(2 phi r) (DLMF 13.14).

Methods (each published, restated here in numpy):

* Steed's method: CF1 for f = F'/F from the l-recurrence (A&S 14.2.1-3), CF2
  for p + iq = (G' + iF')/(G + iF), and the Wronskian for the normalisation
  (Barnett, Feng, Steed & Goldfarb, Comput. Phys. Commun. 8 (1974) 377;
  Barnett, CPC 27 (1982) 147).  CF2 needs about 4|eta| terms, so for
  |eta| > ETA_STEED (channels within (z/ETA_STEED)^2 Ry of threshold) the
  oracle calls mpmath's arbitrary-precision coulombf/coulombg instead and
  forms the derivatives from A&S 14.2.2.
* Closed channels with kappa <= KAPPA_CF: the continued fraction for
  W_{kappa-1}/W_kappa that follows from the kappa-recurrence of W (DLMF
  13.15.1), with the derivative from
  x W'(x) = (kappa - x/2) W + ((kappa - 1/2)^2 - mu^2) W_{kappa-1}.
  Its forward evaluation loses accuracy for larger kappa (weakly closed
  channels), where the oracle calls mpmath.whitw for W_kappa and W_{kappa-1}.
"""
import math

import mpmath
import numpy as np

ETA_STEED = 100.0      # |eta| above this: mpmath Coulomb functions
KAPPA_CF = 8.0         # kappa above this: mpmath Whittaker functions
_TINY = 1e-150   # Lentz zero-guard; small enough, and its square stays finite
_MP_DPS = 30


def _cf1(L, eta, rho, tol=1e-16, maxit=200000):
    """f = F_L'/F_L by modified Lentz on A&S 14.2.1-2 and the sign of F_L.

    With S_m = m/rho + eta/m and R_m^2 = 1 + eta^2/m^2, the l-recurrence gives
    f_L = S_{L+1} - R_{L+1}^2 / (S_{L+1} + S_{L+2} - R_{L+2}^2 / (...)).
    Every negative Lentz denominator marks a sign change of F between
    consecutive l (the tails equal R_m F_{m-1}/F_m), and F_l > 0 for l >> rho.
    """
    L = L.astype(np.float64)
    S1 = (L + 1.0) / rho + eta / (L + 1.0)
    f = np.where(S1 == 0.0, _TINY, S1)
    C = f.copy()
    D = np.zeros_like(f)
    sgn = np.ones_like(f)
    done = np.zeros(f.shape, dtype=bool)
    for j in range(1, maxit):
        m = L + j
        a = -(1.0 + (eta / m) ** 2)
        b = (m / rho + eta / m) + ((m + 1.0) / rho + eta / (m + 1.0))
        Dn = b + a * D
        Dn = np.where(Dn == 0.0, _TINY, Dn)
        Cn = b + a / C
        Cn = np.where(Cn == 0.0, _TINY, Cn)
        Dn = 1.0 / Dn
        delta = Cn * Dn
        live = ~done
        f = np.where(live, f * delta, f)
        sgn = np.where(live & (Dn < 0.0), -sgn, sgn)
        C = np.where(live, Cn, C)
        D = np.where(live, Dn, D)
        done = done | (np.abs(delta - 1.0) < tol)
        if done.all():
            break
    else:
        raise RuntimeError("CF1 did not converge")
    return f, sgn


def _cf2(L, eta, rho, tol=1e-16, maxit=200000):
    """p + iq = H'/H with H = G + iF (Steed's CF2).

    H'/H = i(1 - eta/rho) + (i/rho) a_1/(b_1 + a_2/(b_2 + ...)) with
    a_k = (i eta - L + k - 1)(i eta + L + k), b_k = 2(rho - eta) + 2ik.
    Summed as a series of convergent differences.
    """
    L = L.astype(np.float64)
    a = (-(eta * eta + L * (L + 1.0))) + 1j * eta
    b = 2.0 * (rho - eta) + 2.0j
    pq = 1j * (1.0 - eta / rho)
    D = 1.0 / b
    dH = (1j / rho) * a * D
    pq = pq + dH
    done = np.abs(dH) < tol * np.abs(pq)
    for k in range(1, maxit):
        if done.all():
            break
        a = a + (2.0 * k + 2.0j * eta)
        b = b + 2.0j
        D = 1.0 / (a * D + b)
        dH = (b * D - 1.0) * dH
        live = ~done
        pq = np.where(live, pq + dH, pq)
        done = done | (np.abs(dH) < tol * np.abs(pq))
    else:
        raise RuntimeError("CF2 did not converge")
    return pq.real, pq.imag


def _coulomb_mp(L, eta, rho):
    """F, F', G, G' from mpmath (arbitrary precision), derivatives by A&S 14.2.2."""
    with mpmath.workdps(_MP_DPS):
        e = mpmath.mpf(float(eta))
        r = mpmath.mpf(float(rho))
        F0 = mpmath.coulombf(L, e, r)
        G0 = mpmath.coulombg(L, e, r)
        F1 = mpmath.coulombf(L + 1, e, r)
        G1 = mpmath.coulombg(L + 1, e, r)
        S = (L + 1) / r + e / (L + 1)
        R = mpmath.sqrt((L + 1) ** 2 + e * e) / (L + 1)
        Fp = S * F0 - R * F1
        Gp = S * G0 - R * G1
        return float(F0), float(Fp), float(G0), float(Gp)


def coulomb_fg(l, eta, rho):
    """Coulomb F_l, dF/drho, G_l, dG/drho (DLMF 33.2), element-wise, FP64.

    ``l`` integer >= 0, ``eta`` real, ``rho`` > 0; arrays broadcast together.
    Accurate to ~1e-13 beyond the turning point rho > eta + sqrt(eta^2 +
    l(l+1)), where CF2 converges; at the boundary r = a of an attractive
    (z > 0) ion this holds for every k whenever 2 z a > l(l+1).
    """
    l, eta, rho = np.broadcast_arrays(np.asarray(l, dtype=np.int64),
                                      np.asarray(eta, dtype=np.float64),
                                      np.asarray(rho, dtype=np.float64))
    shape = l.shape
    l, eta, rho = l.ravel(), eta.ravel(), rho.ravel()
    F = np.empty(l.shape)
    Fp = np.empty(l.shape)
    G = np.empty(l.shape)
    Gp = np.empty(l.shape)
    st = np.abs(eta) <= ETA_STEED
    if st.any():
        f, sgn = _cf1(l[st], eta[st], rho[st])
        p, q = _cf2(l[st], eta[st], rho[st])
        # Wronskian F'G - FG' = 1 with G = (f - p) F / q, G' = p G - q F
        Fs = sgn * np.sqrt(q / ((f - p) ** 2 + q * q))
        Gs = (f - p) * Fs / q
        F[st] = Fs
        Fp[st] = f * Fs
        G[st] = Gs
        Gp[st] = p * Gs - q * Fs
    for idx in np.nonzero(~st)[0]:
        F[idx], Fp[idx], G[idx], Gp[idx] = _coulomb_mp(int(l[idx]), eta[idx],
                                                       rho[idx])
    return (F.reshape(shape), Fp.reshape(shape), G.reshape(shape),
            Gp.reshape(shape))


def open_channel_functions(l, z, k, a):
    """s, c, s', c' at r = a for open channels (energy-normalised form).

    s = k^{-1/2} F_l(eta, ka), c = k^{-1/2} G_l(eta, ka), s' = ds/dr =
    k^{1/2} F_l', c' = k^{1/2} G_l', eta = -z/k.  The Wronskian is
    c s' - s c' = 1, so the K-matrix they define is symmetric.
    """
    k = np.asarray(k, dtype=np.float64)
    eta = -float(z) / k
    F, Fp, G, Gp = coulomb_fg(l, eta, k * a)
    sk = np.sqrt(k)
    return F / sk, G / sk, Fp * sk, Gp * sk


def _whittaker_cf(kappa, mu, x, tol=1e-16, maxit=2000000):
    """W_{kappa-1,mu}(x)/W_{kappa,mu}(x) by modified Lentz.

    From W_{k+1} + (2k - x) W_k + ((k - 1/2)^2 - mu^2) W_{k-1} = 0
    (DLMF 13.15.1), r_k = W_{k-1}/W_k = 1/(b_1 - c_{k-1}/(b_2 - c_{k-2}/...))
    with b_j = x + 2j - 2 kappa and c_m = (m - 1/2)^2 - mu^2.  W is the
    minimal solution as kappa decreases; convergence is only tested once j
    has passed kappa + mu, where the recurrence stops changing character.
    """
    f = np.full(kappa.shape, _TINY)
    C = f.copy()
    D = np.zeros_like(f)
    jmin = kappa + mu + 2.0
    nok = np.zeros(kappa.shape, dtype=np.int64)
    done = np.zeros(kappa.shape, dtype=bool)
    for j in range(1, maxit):
        if j == 1:
            a = np.ones_like(f)
        else:
            m = kappa - (j - 1)
            a = -((m - 0.5) ** 2 - mu * mu)
        b = x + 2.0 * j - 2.0 * kappa
        Dn = b + a * D
        Dn = np.where(Dn == 0.0, _TINY, Dn)
        Cn = b + a / C
        Cn = np.where(Cn == 0.0, _TINY, Cn)
        Dn = 1.0 / Dn
        delta = Cn * Dn
        live = ~done
        f = np.where(live, f * delta, f)
        C = np.where(live, Cn, C)
        D = np.where(live, Dn, D)
        ok = (j > jmin) & (np.abs(delta - 1.0) < tol)
        nok = np.where(ok, nok + 1, 0)
        done = done | (nok >= 3)
        if done.all():
            break
    else:
        raise RuntimeError("Whittaker CF did not converge")
    return f


def _whittaker_logderiv_mp(kappa, mu, x):
    with mpmath.workdps(_MP_DPS):
        k = mpmath.mpf(float(kappa))
        m = mpmath.mpf(float(mu))
        xx = mpmath.mpf(float(x))
        W = mpmath.whitw(k, m, xx)
        Wm = mpmath.whitw(k - 1, m, xx)
        return float(k - xx / 2 + ((k - 0.5) ** 2 - m * m) * Wm / W)


def closed_channel_logderiv(l, z, phi, a):
    """L = a W'(a)/W(a) for W(r) = W_{kappa, l+1/2}(2 phi r), kappa = z/phi.

    W decays as exp(-phi r) (DLMF 13.14.21), the bound-state-like solution of
    u'' = [phi^2 + l(l+1)/r^2 - 2z/r] u.  With x = 2 phi a,
    L = x W'(x)/W(x) = kappa - x/2 + ((kappa-1/2)^2 - mu^2) W_{kappa-1}/W_kappa.
    """
    l, phi = np.broadcast_arrays(np.asarray(l, dtype=np.int64),
                                 np.asarray(phi, dtype=np.float64))
    shape = l.shape
    l, phi = l.ravel(), phi.ravel()
    kappa = float(z) / phi
    mu = l + 0.5
    x = 2.0 * phi * a
    out = np.empty(l.shape)
    cf = kappa <= KAPPA_CF
    if cf.any():
        r = _whittaker_cf(kappa[cf], mu[cf], x[cf])
        kc = kappa[cf]
        out[cf] = kc - x[cf] / 2.0 + ((kc - 0.5) ** 2 - mu[cf] ** 2) * r
    for idx in np.nonzero(~cf)[0]:
        out[idx] = _whittaker_logderiv_mp(kappa[idx], mu[idx], x[idx])
    return out.reshape(shape)


def _selftest():  # pragma: no cover - quick manual check
    F, Fp, G, Gp = coulomb_fg(0, 0.0, 1.3)
    assert abs(F - math.sin(1.3)) < 1e-14 and abs(G - math.cos(1.3)) < 1e-14
