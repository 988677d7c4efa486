// Channel functions at the R-matrix boundary r = a, FP64 device code.
//
// Open channel (E > e_i): Coulomb F_l(eta, rho), G_l(eta, rho) and their
// rho-derivatives at rho = k a, eta = -z/k, by Steed's method: CF1 gives
// F'/F from the l-recurrence (Abramowitz & Stegun 14.2.1-2), CF2 gives
// (G' + iF')/(G + iF) (Barnett et al., Comput. Phys. Commun. 8 (1974) 377;
// Barnett, CPC 27 (1982) 147), and the Wronskian F'G - FG' = 1 fixes the
// normalisation.  Returned in energy normalisation s = F/sqrt(k),
// c = G/sqrt(k), s' = sqrt(k) F', c' = sqrt(k) G' (primes d/dr).
//
// Closed channel (E < e_i): the decaying Whittaker function
// W_{kappa, l+1/2}(x), x = 2 phi r, phi = sqrt(e_i - E), kappa = z/phi
// (DLMF 13.14).  Only the pair (W, a dW/dr) up to a common factor enters the
// matching; it is returned scaled to unit length.  Two evaluations:
//  * kappa small: continued fraction for W_{kappa-1}/W_kappa from the
//    kappa-recurrence (DLMF 13.15.1), with
//    x W'(x) = (kappa - x/2) W + ((kappa - 1/2)^2 - mu^2) W_{kappa-1};
//  * kappa large (weakly closed channel, x small): W = exp(-x/2) x^(l+1)
//    U(l+1-kappa, 2l+2, x) with Tricomi's U in its logarithmic series for
//    integer b (DLMF 13.2.9), multiplied through by Gamma(a) sin(pi kappa) so
//    that Rydberg poles (integer kappa) stay finite; the digamma reflection
//    psi(1-y) - psi(y) = pi cot(pi y) produces the pi cos(pi kappa) term.
#pragma once

#include <hip/hip_runtime.h>

namespace rmx {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kLentzTiny = 1e-150;
constexpr double kCfTol = 1e-15;
constexpr int kCf1MaxIt = 100000;
constexpr int kCf2MaxIt = 400000;
constexpr int kWhitMaxIt = 200000;

struct OpenVals {
  double s, c, sp, cp;
  int ok;
};

__device__ inline OpenVals coulomb_open(int L, double z, double k, double a) {
  const double eta = -z / k;
  const double rho = k * a;
  const double Lf = (double)L;
  OpenVals r;
  r.ok = 1;
  // CF1: f = S_{L+1} - R^2_{L+1}/(T_{L+1} - R^2_{L+2}/(T_{L+2} - ...)),
  // S_m = m/rho + eta/m, R_m^2 = 1 + (eta/m)^2, T_m = S_m + S_{m+1}.
  double f = (Lf + 1.0) / rho + eta / (Lf + 1.0);
  if (f == 0.0) f = kLentzTiny;
  double C = f, D = 0.0, sgn = 1.0;
  double Sm = f;  // S_{L+1}
  for (int j = 1;; ++j) {
    const double m = Lf + j;
    const double Sn = (m + 1.0) / rho + eta / (m + 1.0);
    const double em = eta / m;
    const double av = -(1.0 + em * em);
    const double b = Sm + Sn;
    Sm = Sn;
    D = b + av * D;
    if (D == 0.0) D = kLentzTiny;
    C = b + av / C;
    if (C == 0.0) C = kLentzTiny;
    D = 1.0 / D;
    const double delta = C * D;
    f *= delta;
    if (D < 0.0) sgn = -sgn;
    if (fabs(delta - 1.0) < kCfTol) break;
    if (j >= kCf1MaxIt) { r.ok = 0; break; }
  }
  // CF2: p + iq = i(1 - eta/rho) + (i/rho) a_1/(b_1 + a_2/(b_2 + ...)),
  // a_k = (i eta - L + k - 1)(i eta + L + k), b_k = 2(rho - eta) + 2ik,
  // summed as differences of successive convergents.
  double ar = -(eta * eta + Lf * (Lf + 1.0)), ai = eta;
  double br = 2.0 * (rho - eta), bi = 2.0;
  double den = br * br + bi * bi;
  double Dr = br / den, Di = -bi / den;  // D = 1/b
  // dH = (i/rho) * a * D
  double tr = ar * Dr - ai * Di, ti = ar * Di + ai * Dr;
  double hr = -ti / rho, hi = tr / rho;
  double p = hr, q = (1.0 - eta / rho) + hi;
  for (int kk = 1;; ++kk) {
    ar += 2.0 * kk;
    ai += 2.0 * eta;
    bi += 2.0;
    // D = 1/(a D + b)
    const double xr = ar * Dr - ai * Di + br;
    const double xi = ar * Di + ai * Dr + bi;
    den = xr * xr + xi * xi;
    Dr = xr / den;
    Di = -xi / den;
    // dH = (b D - 1) dH
    const double ur = br * Dr - bi * Di - 1.0;
    const double ui = br * Di + bi * Dr;
    const double nr = ur * hr - ui * hi;
    const double ni = ur * hi + ui * hr;
    hr = nr;
    hi = ni;
    p += hr;
    q += hi;
    if (fabs(hr) + fabs(hi) < kCfTol * (fabs(p) + fabs(q))) break;
    if (kk >= kCf2MaxIt) { r.ok = 0; break; }
  }
  // Wronskian normalisation: F^2 = q/((f-p)^2 + q^2), G = (f-p)F/q.
  const double fp = f - p;
  const double F = sgn * sqrt(q / (fp * fp + q * q));
  const double G = fp * F / q;
  const double Fd = f * F;
  const double Gd = p * G - q * F;
  const double sk = sqrt(k);
  r.s = F / sk;
  r.c = G / sk;
  r.sp = Fd * sk;
  r.cp = Gd * sk;
  return r;
}

// psi(y) for y > 0: upward recurrence to y >= 10, then the asymptotic series
// ln y - 1/(2y) - sum_n B_2n / (2n y^2n) through B_14.
__device__ inline double digamma_pos(double y) {
  double acc = 0.0;
  while (y < 10.0) {
    acc -= 1.0 / y;
    y += 1.0;
  }
  const double yi = 1.0 / y, y2 = yi * yi;
  const double ser =
      y2 * (1.0 / 12.0 -
            y2 * (1.0 / 120.0 -
                  y2 * (1.0 / 252.0 -
                        y2 * (1.0 / 240.0 -
                              y2 * (1.0 / 132.0 -
                                    y2 * (691.0 / 32760.0 - y2 / 12.0))))));
  return acc + log(y) - 0.5 * yi - ser;
}

struct ClosedVals {
  double e, ep;  // (W, a W') scaled to unit length
  int ok;
};

// Switch between the continued fraction (accurate for small kappa, worse as
// l grows) and the U series (accurate for small x = 2 z a / kappa).
__device__ inline double whittaker_kappa_switch(int l) {
  const double v = 36.0 - 6.0 * l;
  return v > 8.0 ? v : 8.0;
}

__device__ inline ClosedVals whittaker_cf(int l, double kappa, double x) {
  // r = W_{kappa-1}/W_kappa = 1/(b_1 - c_{kappa-1}/(b_2 - c_{kappa-2}/...)),
  // b_j = x + 2j - 2 kappa, c_m = (m - 1/2)^2 - mu^2; convergence counted
  // only once j is past kappa + mu.
  const double mu = l + 0.5;
  double f = kLentzTiny, C = f, D = 0.0;
  const double jmin = kappa + mu + 2.0;
  int nok = 0;
  ClosedVals out;
  out.ok = 1;
  for (int j = 1;; ++j) {
    double av;
    if (j == 1) {
      av = 1.0;
    } else {
      const double m = kappa - (j - 1) - 0.5;
      av = -(m * m - mu * mu);
    }
    const double b = x + 2.0 * j - 2.0 * kappa;
    D = b + av * D;
    if (D == 0.0) D = kLentzTiny;
    C = b + av / C;
    if (C == 0.0) C = kLentzTiny;
    D = 1.0 / D;
    const double delta = C * D;
    f *= delta;
    if (j > jmin && fabs(delta - 1.0) < kCfTol) {
      if (++nok >= 3) break;
    } else {
      nok = 0;
    }
    if (j >= kWhitMaxIt) { out.ok = 0; break; }
  }
  const double km = kappa - 0.5;
  // (W, x W') ~ (1, kappa - x/2 + c_kappa r); x W'(x) equals a dW/dr at r = a
  const double d1 = 1.0;
  const double d2 = kappa - 0.5 * x + (km * km - mu * mu) * f;
  const double nrm = hypot(d1, d2);
  out.e = d1 / nrm;
  out.ep = d2 / nrm;
  return out;
}

__device__ inline ClosedVals whittaker_useries(int l, double kappa, double x) {
  const int n = 2 * l + 1;
  const double a = l + 1.0 - kappa;
  const double N = rint(kappa);
  const double frac = kappa - N;  // exact
  const double par = (fmod(fabs(N), 2.0) == 1.0) ? -1.0 : 1.0;
  const double sn = par * sin(kPi * frac);
  const double cs = par * cos(kPi * frac);
  // prefactor (-1)^(n+1) (a-n)_n / n!
  double pref = (n % 2 == 1) ? 1.0 : -1.0;
  for (int j = 1; j <= n; ++j) pref *= (a - j) / j;
  const double lnx = log(x);
  // incremental digammas: psi(1+k), psi(n+1+k)
  double psi1 = -kEulerGamma;
  double psin = -kEulerGamma;
  for (int j = 1; j <= n; ++j) psin += 1.0 / j;
  // psi(a+k) term: reflected (y = kappa - l - k) while a + k < 1/2
  bool reflected = (a < 0.5);
  double psia = reflected ? digamma_pos(kappa - l) : digamma_pos(a);
  double t = 1.0, S = 0.0, Sp = 0.0, big = 0.0;
  ClosedVals out;
  out.ok = 1;
  int small_run = 0;
  for (int k = 0; k < 4000; ++k) {
    const double ak = a + k;
    if (reflected && ak >= 0.5) {
      reflected = false;
      psia = digamma_pos(ak);
    }
    const double spsia = reflected ? (sn * psia + kPi * cs) : sn * psia;
    const double cc = sn * (lnx - psi1 - psin) + spsia;
    const double term = t * cc;
    S += term;
    Sp += t * (k * cc + sn) / x;
    const double at = fabs(term);
    if (at > big) big = at;
    if (k > n + 4 && at <= 1e-17 * fabs(S) && fabs(t) < 1e-30 + 1e-17 * fabs(S)) {
      if (++small_run >= 2) break;
    } else {
      small_run = 0;
    }
    // advance: t_{k+1} = t_k (a+k) x / ((n+1+k)(k+1))
    t *= ak * x / ((n + 1.0 + k) * (k + 1.0));
    psi1 += 1.0 / (k + 1.0);
    psin += 1.0 / (n + 1.0 + k);
    if (reflected) {
      // y_k = kappa - l - k decreases by one: psi(y - 1) = psi(y) - 1/(y - 1)
      psia -= 1.0 / (kappa - l - k - 1.0);
    } else {
      psia += 1.0 / ak;
    }
    if (k == 3999) out.ok = 0;
  }
  double U = pref * S, Ud = pref * Sp;
  big *= fabs(pref);
  // finite part: sum_{k=1}^{n} (k-1)! (1-a+k)_{n-k} / (n-k)! x^-k, times sin
  double fk = 1.0;  // (k-1)!
  double xk = 1.0 / x;
  for (int k = 1; k <= n; ++k) {
    double poch = 1.0;
    for (int j = 0; j < n - k; ++j) poch *= (1.0 - a + k + j) / (j + 1.0);
    const double coef = sn * fk * poch;  // (n-k)! folded into poch
    U += coef * xk;
    Ud += -k * coef * xk / x;
    if (fabs(coef * xk) > big) big = fabs(coef * xk);
    fk *= k;
    xk /= x;
  }
  if (!(big <= 1e11 * fabs(U))) out.ok = 0;  // cancellation ate the digits
  // W = exp(-x/2) x^(l+1) U:  x W'/W = l + 1 - x/2 + x U'/U
  // sign convention: W(a) > 0 (or a W'(a) > 0 where W(a) = 0)
  const double sg = (U > 0.0 || (U == 0.0 && Ud > 0.0)) ? 1.0 : -1.0;
  const double d1 = sg * U;
  const double d2 = sg * ((l + 1.0 - 0.5 * x) * U + x * Ud);
  const double nrm = hypot(d1, d2);
  out.e = d1 / nrm;
  out.ep = d2 / nrm;
  return out;
}

__device__ inline ClosedVals whittaker_closed(int l, double z, double phi,
                                              double a) {
  const double kappa = z / phi;
  const double x = 2.0 * phi * a;
  if (kappa <= whittaker_kappa_switch(l)) return whittaker_cf(l, kappa, x);
  return whittaker_useries(l, kappa, x);
}

}  // namespace rmx
