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
    // Kb = O^T (X O)
    wave_gemm<2>(Aug + n, ld, Aug, ld, O, n, n, n, n);
    wave_gemm<2, G_TA>(Kb, n, O, n, Aug + n, ld, n, n, n);
    if (t == S.n_sec) break;
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
        x[u] = in ? Kb[(int64_t)j * n + i] : 0.0;
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

// Outer-region propagation of every symmetry that has sectors, one
// wavefront per energy, before the matching kernel: R(a) -> R(A) in place.
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
