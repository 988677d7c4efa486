// Matching, K-matrix, T-matrix and collision strengths, one workgroup per
// energy.
//
// With channels sorted by threshold the open channels at energy E are the
// prefix P = [0, n_o).  For each open channel j the solution has open parts
// s_i d_ij + c_i K_ij and closed parts e_i X_ij; the R-matrix relation
// u(a) = R a u'(a) becomes the linear system
//     (D1 - R D2) [K; X] = R[:, P] diag(a s'_P) - [diag(s_P); 0]
// with D1 = diag(c_P, e_Q), D2 = diag(a c'_P, a e'_Q) -- no division by any
// channel function.  Then, with K symmetrised,
//     (1 + K^2) Y = K,  Q = K Y,  T = 2(X - 1) + 2iY, X = (1 + K^2)^-1
// so |T_ij|^2 = 4 (Y_ij^2 + Q_ij^2), and
//     Omega(t, u) += (g/2) sum_{i in t, j in u, open} |T_ij|^2.
//
// Dense algebra runs out of a per-energy global workspace (row-major,
// leading dimension 2n) with a blocked right-looking LU (panels of 16
// columns, partial pivoting) whose trailing updates and products are 64 x 64
// tiles staged through LDS and multiplied on the FP64 matrix cores.
//
// One workgroup owns one energy and loops over every symmetry: it computes
// that symmetry's channel functions, solves, and adds into the energy's
// Omega row, which no other workgroup touches (deterministic, no atomics).
// With a counter the grid is persistent and pulls energies from it.
#include <algorithm>

#include "chanfn.h"
#include "rm_internal.h"

namespace rmx {

constexpr int MT = 256;
constexpr int NB = 16;
constexpr int TB = 64;
constexpr int kMaxChanLds = 2048;

struct WgScratch {
  double sL[TB * (NB + 1)];
  double sU[NB * TB];
  double red_v[4];
  int red_i[4];
  int piv[NB];
  int flag;
  double rowbuf[2][NB];
};

// Block-wide argmax of v (ties -> smaller index).
__device__ inline int wg_argmax(double v, int idx, WgScratch &sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  if (lane == 0) {
    sh.red_v[wave] = v;
    sh.red_i[wave] = idx;
  }
  __syncthreads();
  double bv = sh.red_v[0];
  int bi = sh.red_i[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    const double ov = sh.red_v[w];
    const int oi = sh.red_i[w];
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  __syncthreads();
  return bi;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// C (rows x cols) op= A (rows x kd) * B (kd x cols), all in global memory.
// mode 0: C -= AB;  mode 1: C = AB + I;  mode 2: C = AB.
// 64 x 64 output tiles; A and B are staged in LDS 16 columns/rows at a
// time and multiplied on the FP64 matrix cores (16x16x4): each wave owns a
// 32 x 32 quarter of the tile as 2 x 2 MFMA blocks.
__device__ void wg_gemm(double *C, int ldc, const double *A, int lda,
                        const double *B, int ldb, int rows, int cols, int kd,
                        int mode, WgScratch &sh) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  for (int rb = 0; rb < rows; rb += TB) {
    for (int cb = 0; cb < cols; cb += TB) {
      d4 acc[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < kd; k0 += NB) {
        for (int idx = tid; idx < TB * NB; idx += MT) {
          const int r = idx / NB, k = idx % NB;
          sh.sL[r * (NB + 1) + k] = (rb + r < rows && k0 + k < kd)
                                        ? A[(int64_t)(rb + r) * lda + k0 + k]
                                        : 0.0;
          const int kk = idx / TB, c = idx % TB;
          sh.sU[kk * TB + c] = (k0 + kk < kd && cb + c < cols)
                                   ? B[(int64_t)(k0 + kk) * ldb + cb + c]
                                   : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < NB; kk += 4) {
          const int kr = kk + kq;
          const double a0 = sh.sL[(wi + col) * (NB + 1) + kr];
          const double a1 = sh.sL[(wi + 16 + col) * (NB + 1) + kr];
          const double b0 = sh.sU[kr * TB + wj + col];
          const double b1 = sh.sU[kr * TB + wj + 16 + col];
          acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
      }
      // FP64 16x16x4 result: D[i][j] at j = lane % 16, i = lane / 16 + 4 r
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = rb + wi + 16 * x + kq + 4 * r;
            const int j = cb + wj + 16 * y + col;
            if (i >= rows || j >= cols) continue;
            double *cp = C + (int64_t)i * ldc + j;
            const double v = acc[x][y][r];
            if (mode == 0)
              *cp -= v;
            else if (mode == 1)
              *cp = v + (i == j ? 1.0 : 0.0);
            else
              *cp = v;
          }
    }
  }
  __syncthreads();
}

// Panel factorisation with partial pivoting, rows [j0, na), columns
// [j0, j0 + jb), straight in global memory (any height).  Records the
// pivot rows in sh.piv and sets sh.flag on an exactly zero pivot.
__device__ void panel_global(double *A, int na, int ld, int j0, int jb,
                             WgScratch &sh) {
  const int tid = threadIdx.x;
  for (int jj = 0; jj < jb; ++jj) {
    const int col = j0 + jj;
    double best = -1.0;
    int bi = na;
    for (int r = col + tid; r < na; r += MT) {
      const double v = fabs(A[(int64_t)r * ld + col]);
      if (v > best) {
        best = v;
        bi = r;
      }
    }
    const int pr = wg_argmax(best, bi, sh);
    if (tid == 0) sh.piv[jj] = pr;
    if (pr != col && tid < jb) {
      double *x = A + (int64_t)col * ld + j0 + tid;
      double *y = A + (int64_t)pr * ld + j0 + tid;
      const double t = *x;
      *x = *y;
      *y = t;
    }
    __syncthreads();
    const double piv = A[(int64_t)col * ld + col];
    if (piv == 0.0 && tid == 0) sh.flag = 1;
    const double inv = 1.0 / piv;
    for (int r = col + 1 + tid; r < na; r += MT) {
      double *row = A + (int64_t)r * ld;
      const double lv = row[col] * inv;
      row[col] = lv;
      const double *prow = A + (int64_t)col * ld;
      for (int c = col + 1; c < j0 + jb; ++c) row[c] = fma(-lv, prow[c], row[c]);
    }
    __syncthreads();
  }
}

// Same factorisation for panels of at most 2*MT rows, held in registers:
// thread t owns local rows t and t + MT; the pivot row is exchanged and
// broadcast through LDS, so a column costs a few barriers and no global
// memory round trip.
__device__ void panel_regs(double *A, int na, int ld, int j0, int jb,
                           WgScratch &sh) {
  const int tid = threadIdx.x;
  const int m = na - j0;
  double v[2][NB];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int rl = tid + q * MT;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      v[q][c] = (rl < m && c < jb) ? A[(int64_t)(j0 + rl) * ld + j0 + c] : 0.0;
  }
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) {
    if (jj >= jb) break;
    double best = -1.0;
    int bi = na;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int rl = tid + q * MT;
      if (rl < m && rl >= jj) {
        const double a = fabs(v[q][jj]);
        if (a > best) {
          best = a;
          bi = j0 + rl;
        }
      }
    }
    const int pr = wg_argmax(best, bi, sh);
    const int prl = pr - j0;
    // owner of the pivot row publishes it; owner of row jj publishes its own
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (tid + q * MT == prl) {
#pragma unroll
        for (int c = 0; c < NB; ++c) sh.rowbuf[0][c] = v[q][c];
      }
    }
    if (tid == jj) {
#pragma unroll
      for (int c = 0; c < NB; ++c) sh.rowbuf[1][c] = v[0][c];
    }
    if (tid == 0) sh.piv[jj] = pr;
    __syncthreads();
    if (prl != jj) {
      if (tid == jj) {
#pragma unroll
        for (int c = 0; c < NB; ++c) v[0][c] = sh.rowbuf[0][c];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (tid + q * MT == prl) {
#pragma unroll
          for (int c = 0; c < NB; ++c) v[q][c] = sh.rowbuf[1][c];
        }
      }
    }
    const double piv = sh.rowbuf[0][jj];
    if (piv == 0.0 && tid == 0) sh.flag = 1;
    const double inv = 1.0 / piv;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int rl = tid + q * MT;
      if (rl < m && rl > jj) {
        const double lv = v[q][jj] * inv;
        v[q][jj] = lv;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c > jj) v[q][c] = fma(-lv, sh.rowbuf[0][c], v[q][c]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int rl = tid + q * MT;
    if (rl < m) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < jb) A[(int64_t)(j0 + rl) * ld + j0 + c] = v[q][c];
    }
  }
  __syncthreads();
}

// Solve A X = B in place for the na x na matrix in columns [0, na) of rows
// [0, na) (leading dimension ld) with right-hand sides in columns
// [na, na + nrhs).  On return the RHS columns hold X.  Returns nonzero if a
// pivot was exactly zero.
__device__ int wg_lu_solve(double *A, int na, int ld, int nrhs,
                           WgScratch &sh) {
  const int tid = threadIdx.x;
  const int ntot = na + nrhs;
  if (tid == 0) sh.flag = 0;
  __syncthreads();
  for (int j0 = 0; j0 < na; j0 += NB) {
    const int jb = min(NB, na - j0);
    // --- panel factorisation, columns [j0, j0 + jb)
    if (na - j0 <= 2 * MT)
      panel_regs(A, na, ld, j0, jb, sh);
    else
      panel_global(A, na, ld, j0, jb, sh);
    // --- row interchanges and L11^-1 on the columns right of the panel
    for (int c = j0 + jb + tid; c < ntot; c += MT) {
      double x[NB];
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) {
        if (jj < jb) {
          const int pr = sh.piv[jj];
          const int rr = j0 + jj;
          if (pr != rr) {
            double *a = A + (int64_t)rr * ld + c;
            double *b = A + (int64_t)pr * ld + c;
            const double t = *a;
            *a = *b;
            *b = t;
          }
        }
      }
#pragma unroll
      for (int jj = 0; jj < NB; ++jj)
        x[jj] = (jj < jb) ? A[(int64_t)(j0 + jj) * ld + c] : 0.0;
#pragma unroll
      for (int jj = 1; jj < NB; ++jj) {
        if (jj < jb) {
          double s = x[jj];
          const double *lrow = A + (int64_t)(j0 + jj) * ld + j0;
#pragma unroll
          for (int ii = 0; ii < NB; ++ii)
            if (ii < jj) s = fma(-lrow[ii], x[ii], s);
          x[jj] = s;
        }
      }
#pragma unroll
      for (int jj = 0; jj < NB; ++jj)
        if (jj < jb) A[(int64_t)(j0 + jj) * ld + c] = x[jj];
    }
    __syncthreads();
    // --- trailing update
    const int r0 = j0 + jb;
    if (r0 < na) {
      wg_gemm(A + (int64_t)r0 * ld + r0, ld, A + (int64_t)r0 * ld + j0, ld,
              A + (int64_t)j0 * ld + r0, ld, na - r0, ntot - r0, jb, 0, sh);
    }
  }
  // --- back substitution U X = B' on the RHS columns
  for (int j0 = ((na - 1) / NB) * NB; j0 >= 0; j0 -= NB) {
    const int jb = min(NB, na - j0);
    for (int c = na + tid; c < ntot; c += MT) {
      double x[NB];
#pragma unroll
      for (int jj = 0; jj < NB; ++jj)
        x[jj] = (jj < jb) ? A[(int64_t)(j0 + jj) * ld + c] : 0.0;
#pragma unroll
      for (int jj = NB - 1; jj >= 0; --jj) {
        if (jj < jb) {
          const double *urow = A + (int64_t)(j0 + jj) * ld + j0;
          double s = x[jj];
#pragma unroll
          for (int ii = 0; ii < NB; ++ii)
            if (ii > jj && ii < jb) s = fma(-urow[ii], x[ii], s);
          x[jj] = s / urow[jj];
        }
      }
#pragma unroll
      for (int jj = 0; jj < NB; ++jj)
        if (jj < jb) A[(int64_t)(j0 + jj) * ld + c] = x[jj];
    }
    __syncthreads();
    if (j0 > 0) {
      wg_gemm(A + na, ld, A + j0, ld, A + (int64_t)j0 * ld + na, ld, j0, nrhs,
              jb, 0, sh);
    }
  }
  __syncthreads();
  return sh.flag;
}

// Omega(t, u) += 2g sum_{i in t, j in u, i,j < no} (Y_ij^2 + Q_ij^2)
__device__ void accumulate_omega(const SymDev &S, int n_out, const double *Y,
                                 const double *Q, int ld, int no, double *om,
                                 int &nonfinite) {
  const int tid = threadIdx.x;
  const int NT = S.n_target;
  for (int t = 0; t < NT; ++t) {
    const int ta = S.tptr[t], tb = S.tptr[t + 1];
    if (ta == tb || S.tch[ta] >= no) continue;  // lists ascending
    for (int u = t + tid; u < NT; u += MT) {
      const int ua = S.tptr[u], ub = S.tptr[u + 1];
      if (ua == ub || S.tch[ua] >= no) continue;
      double sum = 0.0;
      for (int x = ta; x < tb; ++x) {
        const int i = S.tch[x];
        if (i >= no) break;
        for (int y = ua; y < ub; ++y) {
          const int j = S.tch[y];
          if (j >= no) break;
          const double yv = Y[(int64_t)i * ld + j];
          const double qv = Q[(int64_t)i * ld + j];
          sum += yv * yv + qv * qv;
        }
      }
      sum *= 2.0 * S.g;
      if (!isfinite(sum)) nonfinite = 1;
      om[t * n_out - (t * (t - 1)) / 2 + (u - t)] += sum;
    }
  }
}

// Channel functions of symmetry S at energy Ee into ch[0..n), sorted order.
__device__ int channel_functions(const SymDev &S, double Ee, ChanSlot *ch) {
  int bits = 0;
  for (int i = threadIdx.x; i < S.n; i += MT) {
    const double diff = Ee - S.e_thr[i];
    ChanSlot c;
    if (diff > 0.0) {
      const OpenVals v = coulomb_open(S.l[i], S.z, sqrt(diff), S.a);
      c.d1 = v.c;
      c.d2 = S.a * v.cp;
      c.s = v.s;
      c.asp = S.a * v.sp;
      if (!v.ok) bits |= RM_E_CF_NOCONV;
    } else if (diff < 0.0) {
      const ClosedVals v = whittaker_closed(S.l[i], S.z, sqrt(-diff), S.a);
      c.d1 = v.e;
      c.d2 = v.ep;
      c.s = 0.0;
      c.asp = 0.0;
      if (!v.ok) bits |= RM_E_CF_NOCONV;
    } else {
      c.d1 = 1.0;
      c.d2 = 0.0;
      c.s = 0.0;
      c.asp = 0.0;
      bits |= RM_E_ON_THRESHOLD;
    }
    ch[i] = c;
  }
  return bits;
}

__device__ int count_open(const SymDev &S, double Ee) {
  int lo = 0, hi = S.n;  // thresholds strictly below E
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (S.e_thr[mid] < Ee)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

struct MatchSmem {
  WgScratch sh;
  int rank[kMaxChanLds];
  int bits;
};

// One symmetry at one energy.  Returns RM_E_* bits.
__device__ int match_one(const MatchLaunch &L, int s, int e, MatchSmem &sm) {
  const SymDev &S = L.syms[s];
  const int tid = threadIdx.x;
  const int n = S.n;
  const int ld = 2 * n;
  const double Ee = L.E[e];
  double *Aug = L.work + (int64_t)e * L.work_estride + L.work_off[s];
  double *Kb = Aug + (int64_t)2 * n * n;
  const int no = count_open(S, Ee);
  int stat = 0;
  if (tid == 0) sm.bits = 0;
  __syncthreads();
  if (L.n_open_out && s == 0 && tid == 0) L.n_open_out[e] = no;
  if (no == 0) {
    if (L.K_out && s == 0) {
      double *Ko = L.K_out + (int64_t)e * n * n;
      for (int idx = tid; idx < n * n; idx += MT) Ko[idx] = 0.0;
    }
    __syncthreads();
    return RM_E_NO_OPEN;
  }
  // rank of each open channel among the open channels' input indices
  for (int i = tid; i < no; i += MT) {
    const int pi = S.perm[i];
    int r = 0;
    for (int j = 0; j < no; ++j) r += (S.perm[j] < pi);
    sm.rank[i] = r;
  }
  const bool k_given = (L.K_in != nullptr) && s == 0;
  if (!k_given) {
    ChanSlot *ch = L.chan + (int64_t)e * L.chan_estride + L.chan_off[s];
    const int b = channel_functions(S, Ee, ch);
    if (b) atomicOr(&sm.bits, b);
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += MT) {
      const int i = idx / n, j = idx % n;
      double *a = Aug + (int64_t)i * ld + j;
      const double rij = *a;
      const ChanSlot cj = ch[j];
      *a = (i == j ? ch[i].d1 : 0.0) - rij * cj.d2;
      if (j < no) Aug[(int64_t)i * ld + n + j] = rij * cj.asp - (i == j ? ch[i].s : 0.0);
    }
    __syncthreads();
    if (wg_lu_solve(Aug, n, ld, no, sm.sh)) stat |= RM_E_SINGULAR;
    // K = sym(Z[0:no, 0:no]) -> Kb (ld n)
    for (int idx = tid; idx < no * no; idx += MT) {
      const int i = idx / no, j = idx % no;
      Kb[(int64_t)i * n + j] =
          0.5 * (Aug[(int64_t)i * ld + n + j] + Aug[(int64_t)j * ld + n + i]);
    }
  } else {
    __syncthreads();
    const double *Ki = L.K_in + (int64_t)e * n * n;  // input order, ld n
    for (int idx = tid; idx < no * no; idx += MT) {
      const int i = idx / no, j = idx % no;
      Kb[(int64_t)i * n + j] = Ki[(int64_t)sm.rank[i] * n + sm.rank[j]];
    }
  }
  __syncthreads();
  int nonfinite = 0;
  if (L.K_out && s == 0) {
    double *Ko = L.K_out + (int64_t)e * n * n;
    for (int idx = tid; idx < n * n; idx += MT) {
      const int r = idx / n, c = idx % n;
      if (r >= no || c >= no) Ko[idx] = 0.0;
    }
    for (int idx = tid; idx < no * no; idx += MT) {
      const int i = idx / no, j = idx % no;
      const double v = Kb[(int64_t)i * n + j];
      if (!isfinite(v)) nonfinite = 1;
      Ko[(int64_t)sm.rank[i] * n + sm.rank[j]] = v;
    }
  }
  if (L.do_t) {
    // Pm = 1 + K K in columns [0, no), RHS K in columns [no, 2 no)
    wg_gemm(Aug, ld, Kb, n, Kb, n, no, no, no, 1, sm.sh);
    for (int idx = tid; idx < no * no; idx += MT) {
      const int i = idx / no, j = idx % no;
      Aug[(int64_t)i * ld + no + j] = Kb[(int64_t)i * n + j];
    }
    __syncthreads();
    if (wg_lu_solve(Aug, no, ld, no, sm.sh)) stat |= RM_E_SINGULAR;
    // Q = K Y into columns [0, no)
    wg_gemm(Aug, ld, Kb, n, Aug + no, ld, no, no, no, 2, sm.sh);
    if (L.omega)
      accumulate_omega(S, L.n_target_out, Aug + no, Aug, ld, no,
                       L.omega + (int64_t)e * L.omega_stride, nonfinite);
  }
  if (nonfinite) atomicOr(&sm.bits, RM_E_NONFINITE);
  __syncthreads();
  stat |= sm.bits;
  __syncthreads();
  return stat;
}

__global__ __launch_bounds__(MT) void match_kernel(MatchLaunch L) {
  __shared__ MatchSmem sm;
  __shared__ int s_item;
  const int tid = threadIdx.x;
  int e = blockIdx.x;
  for (;;) {
    if (L.counter) {
      if (tid == 0) s_item = atomicAdd(L.counter, 1);
      __syncthreads();
      e = s_item;
      __syncthreads();
    }
    if (e >= L.m) break;
    int stat = 0;
    for (int s = 0; s < L.n_sym; ++s) stat |= match_one(L, s, e, sm);
    if (tid == 0 && L.status && stat) atomicOr(&L.status[e], stat);
    if (!L.counter) break;
  }
}

hipError_t launch_match(const MatchLaunch &L, hipStream_t st) {
  if (L.m <= 0) return hipSuccess;
  unsigned grid = L.counter ? (unsigned)std::max(1, std::min(L.grid, L.m))
                            : (unsigned)L.m;
  hipLaunchKernelGGL(match_kernel, dim3(grid), dim3(MT), 0, st, L);
  return hipGetLastError();
}

}  // namespace rmx
