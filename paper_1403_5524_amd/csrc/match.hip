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
// columns, partial pivoting) whose trailing updates are register-tiled
// 64 x 64 rank-16 products staged through LDS.
#include "rm_internal.h"

namespace rmx {

constexpr int MT = 256;
constexpr int NB = 16;
constexpr int TB = 64;
constexpr int kMaxChanLds = 2048;

struct WgScratch {
  double sL[TB * NB];
  double sU[NB * TB];
  double red_v[4];
  int red_i[4];
  int piv[NB];
  int flag;
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

// C (rows x cols) op= A (rows x kd) * B (kd x cols), all in global memory.
// mode 0: C -= AB;  mode 1: C = AB + I;  mode 2: C = AB.
__device__ void wg_gemm(double *C, int ldc, const double *A, int lda,
                        const double *B, int ldb, int rows, int cols, int kd,
                        int mode, WgScratch &sh) {
  const int tid = threadIdx.x;
  const int tr = tid >> 4, tc = tid & 15;
  for (int rb = 0; rb < rows; rb += TB) {
    for (int cb = 0; cb < cols; cb += TB) {
      double acc[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[q][p] = 0.0;
      for (int k0 = 0; k0 < kd; k0 += NB) {
        for (int idx = tid; idx < TB * NB; idx += MT) {
          const int r = idx / NB, k = idx % NB;
          sh.sL[idx] = (rb + r < rows && k0 + k < kd)
                           ? A[(int64_t)(rb + r) * lda + k0 + k]
                           : 0.0;
          const int kk = idx / TB, c = idx % TB;
          sh.sU[idx] = (k0 + kk < kd && cb + c < cols)
                           ? B[(int64_t)(k0 + kk) * ldb + cb + c]
                           : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < NB; ++k) {
          double lv[4], uv[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) lv[q] = sh.sL[(tr + 16 * q) * NB + k];
#pragma unroll
          for (int p = 0; p < 4; ++p) uv[p] = sh.sU[k * TB + tc + 16 * p];
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int p = 0; p < 4; ++p) acc[q][p] = fma(lv[q], uv[p], acc[q][p]);
        }
        __syncthreads();
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = rb + tr + 16 * q;
        if (r >= rows) continue;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int c = cb + tc + 16 * p;
          if (c >= cols) continue;
          double *cp = C + (int64_t)r * ldc + c;
          if (mode == 0)
            *cp -= acc[q][p];
          else if (mode == 1)
            *cp = acc[q][p] + (r == c ? 1.0 : 0.0);
          else
            *cp = acc[q][p];
        }
      }
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

struct MatchKArgs {
  const ChanSlot *chan;
  const int32_t *n_open;
  double *work;
  int64_t work_stride;
  int n;
  const int32_t *perm;
  const int32_t *tptr;
  const int32_t *tch;
  int n_target;         // levels of this symmetry
  int n_target_out;     // levels of the omega row
  double g;
  double *K_out;
  double *omega;
  int64_t omega_stride;
  int32_t *status;
  int do_t;
  const double *K_in;   // non-null: skip matching, read K (input order)
};

// Omega(t, u) += 2g sum_{i in t, j in u, i,j < no} (Y_ij^2 + Q_ij^2)
__device__ void accumulate_omega(const MatchKArgs &p, const double *Y,
                                 const double *Q, int ld, int no, double *om,
                                 int &nonfinite) {
  const int tid = threadIdx.x;
  const int NT = p.n_target, NO = p.n_target_out;
  for (int t = 0; t < NT; ++t) {
    const int ta = p.tptr[t], tb = p.tptr[t + 1];
    if (ta == tb || p.tch[ta] >= no) continue;  // lists ascending
    for (int u = t + tid; u < NT; u += MT) {
      const int ua = p.tptr[u], ub = p.tptr[u + 1];
      double sum = 0.0;
      for (int x = ta; x < tb; ++x) {
        const int i = p.tch[x];
        if (i >= no) break;
        for (int y = ua; y < ub; ++y) {
          const int j = p.tch[y];
          if (j >= no) break;
          const double yv = Y[(int64_t)i * ld + j];
          const double qv = Q[(int64_t)i * ld + j];
          sum += yv * yv + qv * qv;
        }
      }
      if (ua < ub && p.tch[ua] < no) {
        sum *= 2.0 * p.g;
        if (!isfinite(sum)) nonfinite = 1;
        om[t * NO - (t * (t - 1)) / 2 + (u - t)] += sum;
      }
    }
  }
}

__global__ __launch_bounds__(MT) void match_kernel(MatchKArgs p) {
  __shared__ WgScratch sh;
  __shared__ int rank[kMaxChanLds];
  __shared__ int s_nonfinite;
  const int tid = threadIdx.x;
  const int e = blockIdx.x;
  const int n = p.n;
  const int ld = 2 * n;
  const int no = p.n_open[e];
  double *Aug = p.work + (int64_t)e * p.work_stride;
  double *Kb = Aug + (int64_t)2 * n * n;
  int stat = 0;
  if (tid == 0) s_nonfinite = 0;
  if (no == 0) {
    if (tid == 0 && p.status) atomicOr(&p.status[e], RM_E_NO_OPEN);
    if (p.K_out) {
      double *Ko = p.K_out + (int64_t)e * n * n;
      for (int idx = tid; idx < n * n; idx += MT) Ko[idx] = 0.0;
    }
    return;
  }
  // rank of each open channel among the open channels' input indices
  for (int i = tid; i < no; i += MT) {
    const int pi = p.perm[i];
    int r = 0;
    for (int j = 0; j < no; ++j) r += (p.perm[j] < pi);
    rank[i] = r;
  }
  __syncthreads();
  if (p.K_in == nullptr) {
    const ChanSlot *ch = p.chan + (int64_t)e * n;
    for (int idx = tid; idx < n * n; idx += MT) {
      const int i = idx / n, j = idx % n;
      double *a = Aug + (int64_t)i * ld + j;
      const double rij = *a;
      const ChanSlot cj = ch[j];
      *a = (i == j ? ch[i].d1 : 0.0) - rij * cj.d2;
      if (j < no) Aug[(int64_t)i * ld + n + j] = rij * cj.asp - (i == j ? ch[i].s : 0.0);
    }
    __syncthreads();
    if (wg_lu_solve(Aug, n, ld, no, sh)) stat |= RM_E_SINGULAR;
    // K = sym(Z[0:no, 0:no]) -> Kb (ld n)
    for (int idx = tid; idx < no * no; idx += MT) {
      const int i = idx / no, j = idx % no;
      Kb[(int64_t)i * n + j] =
          0.5 * (Aug[(int64_t)i * ld + n + j] + Aug[(int64_t)j * ld + n + i]);
    }
  } else {
    const double *Ki = p.K_in + (int64_t)e * n * n;  // input order, ld n
    for (int idx = tid; idx < no * no; idx += MT) {
      const int i = idx / no, j = idx % no;
      Kb[(int64_t)i * n + j] = Ki[(int64_t)rank[i] * n + rank[j]];
    }
  }
  __syncthreads();
  if (p.K_out) {
    double *Ko = p.K_out + (int64_t)e * n * n;
    for (int idx = tid; idx < n * n; idx += MT) {
      const int r = idx / n, c = idx % n;
      if (r >= no || c >= no) Ko[idx] = 0.0;
    }
    for (int idx = tid; idx < no * no; idx += MT) {
      const int i = idx / no, j = idx % no;
      const double v = Kb[(int64_t)i * n + j];
      if (!isfinite(v)) s_nonfinite = 1;
      Ko[(int64_t)rank[i] * n + rank[j]] = v;
    }
  }
  if (p.do_t) {
    // Pm = 1 + K K in columns [0, no), RHS K in columns [no, 2 no)
    wg_gemm(Aug, ld, Kb, n, Kb, n, no, no, no, 1, sh);
    for (int idx = tid; idx < no * no; idx += MT) {
      const int i = idx / no, j = idx % no;
      Aug[(int64_t)i * ld + no + j] = Kb[(int64_t)i * n + j];
    }
    __syncthreads();
    if (wg_lu_solve(Aug, no, ld, no, sh)) stat |= RM_E_SINGULAR;
    // Q = K Y into columns [0, no)
    wg_gemm(Aug, ld, Kb, n, Aug + no, ld, no, no, no, 2, sh);
    if (p.omega) {
      int nf = 0;
      accumulate_omega(p, Aug + no, Aug, ld, no,
                       p.omega + (int64_t)e * p.omega_stride, nf);
      if (nf) s_nonfinite = 1;
    }
  }
  __syncthreads();
  if (s_nonfinite) stat |= RM_E_NONFINITE;
  if (tid == 0 && stat && p.status) atomicOr(&p.status[e], stat);
}

static MatchKArgs make_args(const Sym &s) {
  MatchKArgs k{};
  k.n = s.n;
  k.perm = s.perm;
  k.tptr = s.tptr;
  k.tch = s.tch;
  k.n_target = s.n_target;
  k.g = s.g;
  return k;
}

hipError_t launch_match(const Sym &s, const MatchArgs &a, hipStream_t st) {
  if (a.m <= 0) return hipSuccess;
  if (s.n > kMaxChanLds) return hipErrorInvalidValue;
  MatchKArgs k = make_args(s);
  k.chan = a.chan;
  k.n_open = a.n_open;
  k.work = a.work;
  k.work_stride = a.work_stride;
  k.n_target_out = a.n_target_out;
  k.K_out = a.K_out;
  k.omega = a.omega;
  k.omega_stride = a.omega_stride;
  k.status = a.status;
  k.do_t = a.do_t;
  k.K_in = nullptr;
  hipLaunchKernelGGL(match_kernel, dim3(a.m), dim3(MT), 0, st, k);
  return hipGetLastError();
}

hipError_t launch_t_omega_from_k(const Sym &s, const double *K,
                                 const int32_t *n_open, int64_t m,
                                 double *work, int64_t work_stride,
                                 double *omega, int n_target_out,
                                 hipStream_t st) {
  if (m <= 0) return hipSuccess;
  if (s.n > kMaxChanLds) return hipErrorInvalidValue;
  MatchKArgs k = make_args(s);
  k.n_open = n_open;
  k.work = work;
  k.work_stride = work_stride;
  k.n_target_out = n_target_out;
  k.omega = omega;
  k.omega_stride = (int64_t)n_target_out * (n_target_out + 1) / 2;
  k.do_t = 1;
  k.K_in = K;
  hipLaunchKernelGGL(match_kernel, dim3((unsigned)m), dim3(MT), 0, st, k);
  return hipGetLastError();
}

}  // namespace rmx
