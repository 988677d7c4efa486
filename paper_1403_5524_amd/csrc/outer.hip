// Outer-region propagation kernel.  It has a translation unit of its own so
// that the wavefront linear algebra it shares with the matching kernel (LU,
// GEMM) is compiled separately for each kernel: sharing those routines in
// one unit changed the matching kernel's register allocation.
#define RM_MATCH_DEVICE_ONLY
#include "match.hip"

namespace rmx {

// ---------------------------------------------------------------------------
// Outer-region propagation: the reduced R-matrix X = u u'^-1 = a R(a) is
// carried from a to A through the sectors of S (potential frozen at each
// sector's midpoint): X <- O_s^T X O_s into the sector's eigenbasis, then
//     X <- (c X + s)(c - kappa^2 s X)^-1,  kappa^2 = E - eps,
// c = cos(kappa h), s = sin(kappa h)/kappa (cosh, sinh for kappa^2 < 0),
// exact for a constant potential; finally X <- O^T X O back to the channel
// basis and R(A) = X / A replaces R(a) in Aug's left half.  The step is one
// linear solve, (c - kappa^2 s X)^T Y = (c X + s)^T, Y = X_new^T, set up in
// Aug = [D^T | N^T] for the wavefront LU; X itself lives in Kb.  The
// per-channel c, s, kappa^2 s of a sector go to the channel slots, which
// the channel functions fill only afterwards.  Returns nonzero if a sector
// system was singular.
__device__ int wave_propagate(const SymDev &S, double Ee, double *Aug, int ld,
                              double *Kb, ChanSlot *ch, WaveLds &W) {
  const int lane = lane_id();
  const int n = S.n;
  const int nsq = n * n;
  int flag = 0;
  // X = a R(a) in Aug's left half
  for (int q = lane; q < nsq; q += WT) Aug[(int64_t)(q / n) * ld + q % n] *= S.a;
  wave_sync();
  for (int t = 0; t <= S.n_sec; ++t) {
    const double *O = S.prop_O + (int64_t)t * nsq;
    // Kb = O^T (X O).  X is symmetric, so inside the sectors only the tiles
    // that meet the product's lower triangle are formed and the assembly
    // below reads element (i, j) at (max, min); the final change of basis
    // forms all of it
    wave_gemm_wide<2, 0, 2, 4>(Aug + n, ld, Aug, ld, O, n, n, n, n);
    if (t == S.n_sec) {
      wave_gemm_wide<2, G_TA, 2, 4>(Kb, n, O, n, Aug + n, ld, n, n, n);
      break;
    }
    wave_gemm_wide<2, G_TA | G_LOWER, 2, 4>(Kb, n, O, n, Aug + n, ld, n, n, n);
    const double *eps = S.prop_eps + (int64_t)t * n;
    const double h = S.h_sec;
    for (int i = lane; i < n; i += WT) {
      const double k2 = Ee - eps[i];
      const double k = sqrt(fabs(k2));
      double c, sn;
      if (k2 > 0.0) {
        c = cos(k * h);
        sn = sin(k * h) / k;
      } else if (k2 < 0.0) {
        c = cosh(k * h);
        sn = sinh(k * h) / k;
      } else {
        c = 1.0;
        sn = h;
      }
      ch[i].d1 = c;
      ch[i].d2 = sn;
      ch[i].s = k2 * sn;
    }
    wave_sync();
    // Aug = [(c - kappa^2 s X)^T | (c X + s)^T]
    for (int q0 = lane; q0 < nsq; q0 += UNR * WT) {
      double x[UNR], cj[UNR], sj[UNR], ksj[UNR], ci[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        const bool in = q < nsq;
        const int i = in ? q / n : 0, j = in ? q % n : 0;
        const int hi = i > j ? i : j, lo = i + j - hi;
        x[u] = in ? Kb[(int64_t)hi * n + lo] : 0.0;
        cj[u] = ch[j].d1;
        sj[u] = ch[j].d2;
        ksj[u] = ch[j].s;
        ci[u] = ch[i].d1;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        if (q >= nsq) continue;
        const int i = q / n, j = q % n;
        Aug[(int64_t)i * ld + j] = (i == j ? ci[u] : 0.0) - ksj[u] * x[u];
        Aug[(int64_t)i * ld + n + j] = cj[u] * x[u] + (i == j ? sj[u] : 0.0);
      }
    }
    wave_sync();
    flag |= wave_lu_solve(Aug, n, ld, n, W);
    // X_new = sym(Y^T) into Aug's left half (reads only the right half)
    for (int q0 = lane; q0 < nsq; q0 += UNR * WT) {
      double a[UNR], b[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        const bool in = q < nsq;
        const int i = in ? q / n : 0, j = in ? q % n : 0;
        a[u] = in ? Aug[(int64_t)i * ld + n + j] : 0.0;
        b[u] = in ? Aug[(int64_t)j * ld + n + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        if (q < nsq) Aug[(int64_t)(q / n) * ld + q % n] = 0.5 * (a[u] + b[u]);
      }
    }
    wave_sync();
  }
  // R(A) = X / A into Aug's left half
  const double rA = 1.0 / S.A;
  for (int q = lane; q < nsq; q += WT)
    Aug[(int64_t)(q / n) * ld + q % n] = Kb[q] * rA;
  wave_sync();
  return flag;
}

// ---------------------------------------------------------------------------
// Coupled asymptotic expansion at A (Gailitis).  For the solution that
// behaves as exp(i theta_j) in open channel j, u_i = g_ij exp(i theta_j) with
// g_ij = sum_p d^p_i, d^p = c^p A^-p the terms at r = A.  Collecting powers of
// 1/r in u'' = (W - E) u gives, with br_i(p) = (p + i eta_j - l_i - 1)
// (p + i eta_j + l_i) and V(p) = sum_lam (beta^lam / A^lam) d^(p - lam):
//   e_i != e_j:  d^p_i = [2 i k_j (p-1) d^(p-1)_i - br_i(p-1) d^(p-2)_i / A
//                         + V(p-1)_i] / (A (e_j - e_i)),
//   e_i == e_j:  d^p_i = [br_i(p) d^(p-1)_i / A - V(p)_i] / (2 i k_j p),
// from d^0 = unit column j.  A term is added while its size T_p = max_i
// |d^p_i| does not exceed the previous one (T_0 = 1); the first larger term
// ends the sum unadded, a term at or below kGlConv after adding it.

constexpr double kGlConv = 1e-16;
constexpr double kGlFlag = 1e-6;

// sigma_l(eta) = arg Gamma(l + 1 + i eta): Stirling's series (six terms) at
// w + m0 with Re >= 20, less the arguments of the factors w, ..., w + m0 - 1.
__device__ double coulomb_phase(int l, double eta) {
  const double x0 = l + 1.0;
  const int m0 = x0 < 20.0 ? (int)ceil(20.0 - x0) : 0;
  double sub = 0.0;
  for (int m = 0; m < m0; ++m) sub += atan2(eta, x0 + m);
  const double x = x0 + m0, y = eta;
  const double mod2 = x * x + y * y;
  double im = (x - 0.5) * atan2(y, x) + 0.5 * y * log(mod2) - y;
  const double vr = x / mod2, vi = -y / mod2;              // 1 / w
  const double v2r = vr * vr - vi * vi, v2i = 2.0 * vr * vi;  // 1 / w^2
  const double ck[6] = {1.0 / 12.0,    -1.0 / 360.0, 1.0 / 1260.0,
                        -1.0 / 1680.0, 1.0 / 1188.0, -691.0 / 360360.0};
  double pr = vr, pi = vi;  // 1 / w^(2k - 1)
  for (int k = 0; k < 6; ++k) {
    im += ck[k] * pi;
    const double nr = pr * v2r - pi * v2i, ni = pr * v2i + pi * v2r;
    pr = nr;
    pi = ni;
  }
  return im - sub;
}

__device__ inline int gl_pos(int p, int Q) { return ((-p) % Q + Q) % Q; }

// The matching system at A with the expansion's solutions, in place of the
// one the matching kernel assembles from Coulomb functions: R(A) in Aug's
// left half on entry (copied to Kb), closed channels' functions in ch, the
// open channels j < no in blocks of kGlCols columns (lane l serves column
// l mod kGlCols of a block).  Per block and order one wavefront GEMM forms
// V(p) from the stacked couplings and the doubled ring of earlier orders;
// at the end [A C' | A S'] is multiplied by R for
//   Aug = [C - R A C' | diag(d1_Q) - R_Q diag(d2_Q) | R A S' - S].
// gw: gl_doubles(n, lmax) doubles of scratch.  Returns RM_E_ASYM_NOCONV if
// some channel's first omitted term exceeds kGlFlag.
__device__ int wave_gailitis_system(const SymDev &S, double Ee, double *Aug,
                                    int ld, double *Kb, const ChanSlot *ch,
                                    int no, double *gw) {
  const int lane = lane_id();
  const int n = S.n, nc = n - no;
  const double r = S.A, ir = 1.0 / S.A;
  const int Q = gl_ring(S.lmax);
  constexpr int CB = kGlCols, CW = 2 * kGlCols;
  const int64_t slot = (int64_t)n * CW;
  double *ring = gw;
  double *Vs = ring + 2 * Q * slot;
  double *g = Vs + 2 * slot;
  double *gp = g + slot;
  double *Y = gp + slot;
  double *X = Y + slot;
  int bits = 0;
  wave_copy(Kb, n, Aug, ld, n, n);
  wave_sync();
  for (int q = lane; q < n * nc; q += WT) {
    const int i = q / nc, j = no + q % nc;
    Aug[(int64_t)i * ld + j] =
        (i == j ? ch[j].d1 : 0.0) - Kb[(int64_t)i * n + j] * ch[j].d2;
  }
  const int jj = lane & (CB - 1);
  for (int j0 = 0; j0 < no; j0 += CB) {
    const int j = j0 + jj;
    const bool real_col = j < no;
    const int jc = real_col ? j : 0;
    const double ej = S.e_thr[jc];
    const double kj = real_col ? sqrt(Ee - ej) : 1.0;
    const double eta = -S.z / kj;
    for (int64_t q = lane; q < 2 * Q * slot; q += WT) ring[q] = 0.0;
    for (int64_t q = lane; q < 2 * slot; q += WT) Vs[q] = 0.0;
    for (int64_t q = lane; q < slot; q += WT) {
      g[q] = 0.0;
      gp[q] = 0.0;
    }
    wave_sync();
    if (lane < CB && real_col) {
      const int64_t o = (int64_t)j * CW + jj;
      ring[o] = 1.0;             // order 0 at position 0
      ring[Q * slot + o] = 1.0;  // and its duplicate
      g[o] = 1.0;
    }
    wave_sync();
    bool active = real_col;
    bool ncv = false;
    double t_prev = 1.0;
    for (int P = 1; P <= S.gl_terms; ++P) {
      if (!wave_or(active ? 1 : 0)) break;
      double *Vn = Vs + (P & 1) * slot;
      const double *Vo = Vs + ((P - 1) & 1) * slot;
      const double *d1 = ring + gl_pos(P - 1, Q) * slot;
      const double *d2 = ring + gl_pos(P - 2, Q) * slot;
      double *dn = ring + gl_pos(P, Q) * slot;
      double *dd = dn + Q * slot;
      if (S.lmax > 0)  // V(P): orders P-1 .. P-lmax are consecutive slots
        wave_gemm<2>(Vn, CW, S.gl_beta, S.lmax * n, d1, CW, n, CW,
                     S.lmax * n);
      double tmax = 0.0;
      for (int q = lane; q < n * CB; q += WT) {
        const int i = q / CB;
        const int64_t o = (int64_t)i * CW + jj;
        const double ei = S.e_thr[i];
        const double li = (double)S.l[i];
        const double xr = d1[o], xi = d1[o + CB];
        double nr, ni;
        if (ei == ej) {
          const double a1 = P - li - 1.0, a2 = P + li;
          const double brr = a1 * a2 - eta * eta, bri = eta * (a1 + a2);
          const double ur = (brr * xr - bri * xi) * ir - Vn[o];
          const double ui = (brr * xi + bri * xr) * ir - Vn[o + CB];
          const double f = 1.0 / (2.0 * kj * P);  // u / (2 i k_j P)
          nr = ui * f;
          ni = -ur * f;
        } else {
          const double yr = d2[o], yi = d2[o + CB];
          const double a1 = P - li - 2.0, a2 = P - 1.0 + li;
          const double brr = a1 * a2 - eta * eta, bri = eta * (a1 + a2);
          const double tk = 2.0 * kj * (P - 1);
          const double ur = -tk * xi - (brr * yr - bri * yi) * ir + Vo[o];
          const double ui = tk * xr - (brr * yi + bri * yr) * ir + Vo[o + CB];
          const double f = ir / (ej - ei);
          nr = ur * f;
          ni = ui * f;
        }
        if (!real_col) nr = ni = 0.0;
        dn[o] = nr;
        dn[o + CB] = ni;
        dd[o] = nr;
        dd[o + CB] = ni;
        tmax = fmax(tmax, sqrt(nr * nr + ni * ni));
      }
      tmax = fmax(tmax, __shfl_xor(tmax, 16));
      tmax = fmax(tmax, __shfl_xor(tmax, 32));
      bool add = false;
      if (active) {
        if (tmax > t_prev) {
          active = false;
          ncv = tmax > kGlFlag;
        } else {
          add = true;
          if (tmax <= kGlConv)
            active = false;
          else
            t_prev = tmax;
        }
      }
      if (add) {
        const double m = -P * ir;
        for (int q = lane; q < n * CB; q += WT) {
          const int64_t o = (int64_t)(q / CB) * CW + jj;
          const double nr = dn[o], ni = dn[o + CB];
          g[o] += nr;
          g[o + CB] += ni;
          gp[o] += m * nr;
          gp[o + CB] += m * ni;
        }
      }
      wave_sync();
    }
    if (active) ncv = t_prev > kGlFlag;  // ended at gl_terms terms
    if (ncv) bits |= RM_E_ASYM_NOCONV;
    // u = g e^{i theta} / sqrt(k), u' = (g' + i theta' g) e^{i theta} / sqrt(k)
    const int lj = S.l[jc];
    const double th = kj * r - eta * log(2.0 * kj * r) - 0.5 * M_PI * lj +
                      coulomb_phase(lj, eta);
    const double sq = 1.0 / sqrt(kj);
    const double cr = cos(th) * sq, ci = sin(th) * sq, tp = kj - eta * ir;
    for (int q = lane; q < n * CB; q += WT) {
      const int64_t o = (int64_t)(q / CB) * CW + jj;
      const double gr = g[o], gi = g[o + CB];
      const double hr = gp[o] - tp * gi, hi = gp[o + CB] + tp * gr;
      const double ur = gr * cr - gi * ci, ui = gr * ci + gi * cr;
      const double vr = hr * cr - hi * ci, vi = hr * ci + hi * cr;
      ring[o] = real_col ? ur : 0.0;  // C
      ring[o + CB] = real_col ? ui : 0.0;  // S
      Y[o] = real_col ? r * vr : 0.0;  // A C'
      Y[o + CB] = real_col ? r * vi : 0.0;  // A S'
    }
    wave_sync();
    wave_gemm<2>(X, CW, Kb, n, Y, CW, n, CW, n);
    if (real_col)
      for (int q = lane; q < n * CB; q += WT) {
        const int i = q / CB;
        const int64_t o = (int64_t)i * CW + jj;
        Aug[(int64_t)i * ld + j] = ring[o] - X[o];
        Aug[(int64_t)i * ld + n + j] = X[o + CB] - ring[o + CB];
      }
    wave_sync();
  }
  return bits;
}

// Outer-region propagation of every symmetry that has sectors, one
// wavefront per energy, before the matching kernel: R(a) -> R(A) in place,
// and with the asymptotic expansion the whole matching system at A.
// Sector failures are or-ed into status.
__global__ __launch_bounds__(WT *WPB) void propagate_kernel(MatchLaunch L) {
  __shared__ WaveLds lds[WPB];
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int e = blockIdx.x * WPB + wv;
  if (e >= L.m) return;
  int bits = 0;
  for (int s = 0; s < L.n_sym; ++s) {
    const SymDev &S = L.syms[s];
    if (S.n_sec <= 0) continue;
    double *Aug = L.work + (int64_t)e * L.work_estride + L.work_off[s];
    double *Kb = Aug + (int64_t)2 * S.n * S.n;
    ChanSlot *ch = L.chan + (int64_t)e * L.chan_estride + L.chan_off[s];
    if (wave_propagate(S, L.E[e], Aug, 2 * S.n, Kb, ch, lds[wv]))
      bits |= RM_E_SINGULAR;
    if (S.gl_terms > 0) {
      const int no = count_open(S, L.E[e]);
      if (no > 0) {
        bits |= wave_channel_functions(S, L.E[e], ch);
        wave_sync();
        bits |= wave_gailitis_system(S, L.E[e], Aug, 2 * S.n, Kb, ch, no,
                                     Aug + match_work_doubles(S.n));
      }
    }
  }
  bits = wave_or(bits);
  if (lane == 0 && L.status && bits) atomicOr(&L.status[e], bits);
}

hipError_t launch_propagate(const MatchLaunch &L, hipStream_t st) {
  if (L.m <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((L.m + WPB - 1) / WPB);
  hipLaunchKernelGGL(propagate_kernel, dim3(blocks), dim3(WT * WPB), 0, st, L);
  return hipGetLastError();
}

}  // namespace rmx
