// Post-processing of collision strengths on the energy mesh.
//
// * Gaussian convolution, the smoothing the paper applies before comparing
//   with measurements (Sec. 4 and 5, FWHM of tens of meV):
//       Omega~(E_i) = sum_j g_ij Omega(E_j) / sum_j g_ij,
//       g_ij = exp(-(E_i - E_j)^2 / (2 s^2)) dE_j,  s = FWHM / (2 sqrt(2 ln 2)),
//   dE_j the trapezoid weights of the ascending, possibly non-uniform mesh,
//   the sum cut at |E_i - E_j| <= 8 s; a one-point mesh is left unchanged.
// * Maxwellian-averaged effective collision strengths of each level pair
//   (t, u), upper level e = max(e_t, e_u), outgoing energy eps = E - e:
//       Upsilon(kT) = int_0^inf Omega(eps) exp(-eps/kT) d(eps/kT)
//   with Omega held constant from threshold to the first mesh point above
//   it, the trapezoid rule between mesh points, truncation at the last one.
// * Statistical averaging over the levels of groups (terms): Omega summed
//   over every unordered level pair whose two groups form the group pair.
//
// Omega is energy-major [M][P].  The convolution is a banded matrix product
// Omega~ = G Omega with G normalised row by row; it runs on the FP64 matrix
// cores.  A workgroup owns 64 outputs and 256 transitions, walks the band of
// mesh rows its outputs reach in stages of 16, forms those rows' weights in
// LDS (each exp once per workgroup) beside the staged Omega rows, and every
// wave applies its 16 outputs' weights with 16x16x4 MFMAs.  Upsilon and the
// grouping are single passes over Omega (HBM-bound).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "rm_internal.h"

namespace rmx {

const char *set_error(int code, const char *msg);  // defined in rm_api.hip

static int pp_fail(int code, const std::string &msg) {
  set_error(code, msg.c_str());
  return code;
}

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr double CV_CUT = 8.0;   // kernel cut, in standard deviations
constexpr int CV_BM = 64;        // outputs per workgroup, 16 per wave
constexpr int CV_BP = 256;       // transitions per workgroup
constexpr int CV_NB = CV_BP / 16;
constexpr int CV_KC = 16;        // mesh rows per stage
constexpr int CV_OPAD = 2;       // LDS row padding, doubles

struct CvSmem {
  double O[2][CV_KC][CV_BP + CV_OPAD];
  double W[2][CV_KC][CV_BM + CV_OPAD];
};

__device__ inline int64_t pp_first_ge(const double *E, int64_t m, double x) {
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (E[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}
__device__ inline int64_t pp_first_gt(const double *E, int64_t m, double x) {
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (E[mid] <= x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Trapezoid weights dE, each output's window [lo, hi) and 1 / sum_j g_ij.
__global__ void conv_window_kernel(const double *__restrict__ E, int64_t m,
                                   double s, double r, double *dE, int64_t *lo,
                                   int64_t *hi, double *inv_norm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double Ei = E[i];
  double w = 0.0;
  if (i > 0) w += 0.5 * (Ei - E[i - 1]);
  if (i + 1 < m) w += 0.5 * (E[i + 1] - Ei);
  dE[i] = w;
  const int64_t a = pp_first_ge(E, m, Ei - CV_CUT * s);
  const int64_t b = pp_first_gt(E, m, Ei + CV_CUT * s);
  double sum = 0.0;
  for (int64_t j = a; j < b; ++j) {
    const double x = E[j] - Ei;
    double wj = 0.0;
    if (j > 0) wj += 0.5 * (E[j] - E[j - 1]);
    if (j + 1 < m) wj += 0.5 * (E[j + 1] - E[j]);
    sum += exp(-r * x * x) * wj;
  }
  lo[i] = a;
  hi[i] = b;
  inv_norm[i] = 1.0 / sum;
}

__global__ __launch_bounds__(256) void conv_apply_kernel(
    const double *__restrict__ E, const double *__restrict__ dE, int64_t m,
    const double *__restrict__ in, int64_t P, double r,
    const int64_t *__restrict__ lo, const int64_t *__restrict__ hi,
    const double *__restrict__ inv_norm, double *__restrict__ out,
    int n_tiles) {
  __shared__ CvSmem sm;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // blocks go round-robin over the 8 XCDs: give each XCD a run of
  // consecutive output tiles so their overlapping bands share its L2
  const int per = (n_tiles + 7) / 8;
  const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (tile >= n_tiles) return;
  const int64_t i0 = (int64_t)tile * CV_BM;
  const int64_t ilast = min<int64_t>(i0 + CV_BM, m) - 1;
  const int64_t p0 = (int64_t)blockIdx.y * CV_BP;
  const int nblk = (int)min<int64_t>(CV_NB, (P - p0 + 15) / 16);
  const int64_t jlo = lo[i0], jhi = hi[ilast];

  // this wave's 16 outputs and the rows they reach
  const int64_t wi0 = i0 + 16 * wave;
  const bool wact = wi0 <= ilast;
  const int64_t wlo = wact ? lo[wi0] : 0;
  const int64_t whi = wact ? hi[min<int64_t>(wi0 + 15, ilast)] : 0;

  // weight staging: output i0 + (tid % 64), stage rows tid / 64 + 4 u
  const int si = tid & 63;
  const int sk = tid >> 6;
  const int64_t gi = i0 + si;
  const bool iv = gi <= ilast;
  const double Ei = iv ? E[gi] : 0.0;
  const double ninv = iv ? inv_norm[gi] : 0.0;
  const int64_t ilo = iv ? lo[gi] : 0, ihi = iv ? hi[gi] : 0;
  // Omega staging: column p0 + tid, the 16 rows of a stage
  const int64_t gp = p0 + tid;
  const bool pv = gp < P;

  double rO[CV_KC], rW[4];
  auto fetch = [&](int64_t j0) {
#pragma unroll
    for (int k = 0; k < CV_KC; ++k) {
      const int64_t j = j0 + k;
      rO[k] = (pv && j < jhi) ? in[j * P + gp] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = j0 + sk + 4 * u;
      double w = 0.0;
      if (j >= ilo && j < ihi) {
        const double x = E[j] - Ei;
        w = exp(-r * x * x) * dE[j] * ninv;
      }
      rW[u] = w;
    }
  };
  auto stage = [&](int b) {
#pragma unroll
    for (int k = 0; k < CV_KC; ++k) sm.O[b][k][tid] = rO[k];
#pragma unroll
    for (int u = 0; u < 4; ++u) sm.W[b][sk + 4 * u][si] = rW[u];
  };

  d4 acc[CV_NB];
#pragma unroll
  for (int b = 0; b < CV_NB; ++b) acc[b] = d4{0.0, 0.0, 0.0, 0.0};
  const int kq = lane >> 4;
  const int col = lane & 15;

  fetch(jlo);
  stage(0);
  if (jlo + CV_KC < jhi) fetch(jlo + CV_KC);
  __syncthreads();
  int buf = 0;
  for (int64_t j0 = jlo; j0 < jhi; j0 += CV_KC, buf ^= 1) {
    if (wact && j0 < whi && j0 + CV_KC > wlo) {
#pragma unroll
      for (int kk = 0; kk < CV_KC; kk += 4) {
        const double a = sm.W[buf][kk + kq][16 * wave + col];
#pragma unroll
        for (int b = 0; b < CV_NB; ++b)
          if (b < nblk) {
            const double bv = sm.O[buf][kk + kq][16 * b + col];
            acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[b], 0, 0, 0);
          }
      }
    }
    if (j0 + CV_KC < jhi) {
      stage(buf ^ 1);
      if (j0 + 2 * CV_KC < jhi) fetch(j0 + 2 * CV_KC);
    }
    __syncthreads();
  }

  // FP64 16x16x4 result: lane holds row kq + 4 q, column col of its block
  if (wact) {
#pragma unroll
    for (int b = 0; b < CV_NB; ++b) {
      if (b >= nblk) continue;
      const int64_t p = p0 + 16 * b + col;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t i = wi0 + kq + 4 * q;
        if (i <= ilast && p < P) out[i * P + p] = acc[b][q];
      }
    }
  }
}

__global__ void copy_kernel(const double *__restrict__ in, int64_t n,
                            double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

// exp(-(E_i - E_{i-1}) / kT_t) for i >= 1: f [m][nT]
__global__ void ups_factor_kernel(const double *__restrict__ E, int64_t m,
                                  const double *__restrict__ kT, int nT,
                                  double *f) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m * nT) return;
  const int64_t i = q / nT;
  const int t = (int)(q % nT);
  f[q] = i > 0 ? exp(-(E[i] - E[i - 1]) / kT[t]) : 0.0;
}

constexpr int UP_T = 8;     // temperatures per pass over Omega
constexpr int UP_SEGS = 4;  // mesh segments per workgroup (one per wave)

__device__ inline int64_t wave_min64(int64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int64_t o = __shfl_xor(v, off);
    v = min(v, o);
  }
  return v;
}

// Partial sums over one mesh segment per wave, one transition per lane:
// part [n_seg][P][nT].  exp(-eps/kT) starts exact at each lane's first row
// and then follows the product of the per-interval factors.
__global__ __launch_bounds__(256) void ups_part_kernel(
    const double *__restrict__ E, int64_t m, const double *__restrict__ om,
    int n_target, int64_t P, const double *__restrict__ e_level,
    const double *__restrict__ kT, int nT, const double *__restrict__ f,
    int64_t seg_len, int64_t n_seg, double *__restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t seg = (int64_t)blockIdx.y * UP_SEGS + wave;
  if (seg >= n_seg) return;  // whole wave; no barriers below
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const bool pv = p < P;
  // level pair (t, u), t <= u, of packed index p
  int t = 0;
  int64_t rem = pv ? p : 0;
  while (rem >= n_target - t) {
    rem -= n_target - t;
    ++t;
  }
  const int u = t + (int)rem;
  const double e = pv ? fmax(e_level[t], e_level[u]) : 0.0;
  const int64_t i0 = pv ? pp_first_gt(E, m, e) : m;  // first point above e
  const int64_t s_lo = seg * seg_len;
  const int64_t s_hi = min(m, s_lo + seg_len);
  const int64_t first = pv ? max(i0, s_lo) : m;
  int64_t istart = wave_min64(first);
  istart = ((int64_t)__builtin_amdgcn_readfirstlane((int)(istart >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)istart);

  for (int t0 = 0; t0 < nT; t0 += UP_T) {
    const int nt = min(UP_T, nT - t0);
    double T[UP_T], acc[UP_T], x[UP_T];
#pragma unroll
    for (int q = 0; q < UP_T; ++q) {
      T[q] = q < nt ? kT[t0 + q] : 1.0;
      acc[q] = 0.0;
      x[q] = 0.0;
    }
    for (int64_t i = istart; i < s_hi; ++i) {
      const bool act = i >= first;
      const double v = act ? om[i * P + p] : 0.0;
      const double Ec = E[i];
      const double wr = i + 1 < m ? 0.5 * (E[i + 1] - Ec) : 0.0;
      const double wl = (act && i > i0) ? 0.5 * (Ec - E[i - 1]) : 0.0;
      if (act && i == first) {
#pragma unroll
        for (int q = 0; q < UP_T; ++q) x[q] = exp(-(Ec - e) / T[q]);
        if (i == i0) {  // constant Omega from threshold to E_i0
#pragma unroll
          for (int q = 0; q < UP_T; ++q) acc[q] = v * (1.0 - x[q]);
        }
      } else {
#pragma unroll
        for (int q = 0; q < UP_T; ++q)
          if (q < nt) x[q] *= f[i * nT + t0 + q];
      }
      const double vw = v * (wl + wr);
#pragma unroll
      for (int q = 0; q < UP_T; ++q) acc[q] = fma(vw * x[q], 1.0 / T[q], acc[q]);
    }
    if (pv) {
      double *dst = part + (seg * P + p) * nT + t0;
      for (int q = 0; q < nt; ++q) dst[q] = acc[q];
    }
  }
}

__global__ void ups_reduce_kernel(const double *__restrict__ part,
                                  int64_t n_seg, int64_t n, double *ups) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double s = 0.0;
  for (int64_t g = 0; g < n_seg; ++g) s += part[g * n + q];
  ups[q] = s;
}

// out [m][Pg]: each group pair sums its list of level-pair columns
// (cols[off[q] .. off[q + 1]) of row i); one workgroup per row.
__global__ __launch_bounds__(256) void group_kernel(
    const double *__restrict__ om, int64_t m, int64_t P,
    const int32_t *__restrict__ off, const int32_t *__restrict__ cols,
    int64_t Pg, double *__restrict__ out) {
  for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
    const double *row = om + i * P;
    for (int64_t q = threadIdx.x; q < Pg; q += blockDim.x) {
      double s = 0.0;
      for (int c = off[q]; c < off[q + 1]; ++c) s += row[cols[c]];
      out[i * Pg + q] = s;
    }
  }
}

static int pp_hip(const char *what, hipError_t e) {
  return pp_fail(e == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP,
                 std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace rmx

using namespace rmx;

extern "C" {

int rm_convolve_gaussian(const double *E, int64_t M, const double *omega_in,
                         int64_t P, double fwhm, double *omega_out,
                         void *stream) {
  const char *fn = "rm_convolve_gaussian";
  if (M < 0 || P < 1)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": M < 0 or P < 1");
  if (!(fwhm > 0.0) || !std::isfinite(fwhm))
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": fwhm must be finite and > 0");
  if (M == 0) return RM_OK;
  if (!E || !omega_in || !omega_out)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": null pointer");
  if (omega_in == omega_out)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": in place is not supported");
  hipStream_t st = (hipStream_t)stream;
  if (M == 1) {
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256),
                       0, st, omega_in, P, omega_out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RM_OK : pp_hip(fn, e);
  }
  const int64_t n_tiles = (M + CV_BM - 1) / CV_BM;
  if (n_tiles > (int64_t)1 << 30 || (P + CV_BP - 1) / CV_BP > 65535)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": M or P too large");
  const double s = fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  const double r = 0.5 / (s * s);
  char *ws = nullptr;
  const size_t bytes = (size_t)M * (2 * sizeof(double) + 2 * sizeof(int64_t));
  hipError_t e = hipMallocAsync((void **)&ws, bytes, st);
  if (e != hipSuccess) return pp_hip(fn, e);
  double *dE = (double *)ws;
  double *inv = dE + M;
  int64_t *lo = (int64_t *)(inv + M);
  int64_t *hi = lo + M;
  hipLaunchKernelGGL(conv_window_kernel, dim3((unsigned)((M + 255) / 256)),
                     dim3(256), 0, st, E, M, s, r, dE, lo, hi, inv);
  e = hipGetLastError();
  if (e == hipSuccess) {
    const unsigned gx = (unsigned)(8 * ((n_tiles + 7) / 8));
    const unsigned gy = (unsigned)((P + CV_BP - 1) / CV_BP);
    hipLaunchKernelGGL(conv_apply_kernel, dim3(gx, gy), dim3(256), 0, st, E,
                       dE, M, omega_in, P, r, lo, hi, inv, omega_out,
                       (int)n_tiles);
    e = hipGetLastError();
  }
  const hipError_t ef = hipFreeAsync(ws, st);
  if (e == hipSuccess) e = ef;
  return e == hipSuccess ? RM_OK : pp_hip(fn, e);
}

int rm_effective_collision_strengths(const double *E, int64_t M,
                                     const double *omega, int32_t n_target,
                                     const double *e_level, const double *kT,
                                     int32_t nT, double *upsilon,
                                     void *stream) {
  const char *fn = "rm_effective_collision_strengths";
  if (M < 0 || n_target < 1 || nT < 0)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": M < 0, n_target < 1 or nT < 0");
  if (nT == 0) return RM_OK;
  if (!e_level || !kT || !upsilon)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": null pointer");
  if (M > 0 && (!E || !omega))
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": null E or omega");
  for (int q = 0; q < nT; ++q)
    if (!(kT[q] > 0.0) || !std::isfinite(kT[q]))
      return pp_fail(RM_ERR_ARG, std::string(fn) + ": kT must be finite and > 0");
  for (int t = 0; t < n_target; ++t)
    if (!std::isfinite(e_level[t]))
      return pp_fail(RM_ERR_ARG, std::string(fn) + ": level energy not finite");
  hipStream_t st = (hipStream_t)stream;
  const int64_t P = (int64_t)n_target * (n_target + 1) / 2;
  const int64_t n_col = (P + 63) / 64;
  // enough segments for several thousand waves, none shorter than 128 rows
  int64_t n_seg = std::max<int64_t>(1, std::min<int64_t>((8192 + n_col - 1) / n_col,
                                                         (M + 127) / 128));
  const int64_t seg_len = std::max<int64_t>(1, (M + n_seg - 1) / n_seg);
  n_seg = std::max<int64_t>(1, (M + seg_len - 1) / seg_len);
  if (n_col > 0x7fffffff || (n_seg + UP_SEGS - 1) / UP_SEGS > 65535)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": M or n_target too large");
  const size_t n_part = (size_t)n_seg * P * nT;
  const size_t bytes = sizeof(double) *
      ((size_t)n_target + nT + std::max<size_t>(1, (size_t)M * nT) + n_part);
  char *ws = nullptr;
  hipError_t e = hipMallocAsync((void **)&ws, bytes, st);
  if (e != hipSuccess) return pp_hip(fn, e);
  double *d_lev = (double *)ws;
  double *d_kT = d_lev + n_target;
  double *f = d_kT + nT;
  double *part = f + std::max<int64_t>(1, M * nT);
  e = hipMemcpyAsync(d_lev, e_level, n_target * sizeof(double),
                     hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_kT, kT, nT * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && M > 0) {
    hipLaunchKernelGGL(ups_factor_kernel, dim3((unsigned)((M * nT + 255) / 256)),
                       dim3(256), 0, st, E, M, d_kT, nT, f);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(ups_part_kernel,
                       dim3((unsigned)n_col, (unsigned)((n_seg + UP_SEGS - 1) / UP_SEGS)),
                       dim3(64 * UP_SEGS), 0, st, E, M, omega, n_target, P,
                       d_lev, d_kT, nT, f, seg_len, n_seg, part);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int64_t n = P * nT;
    hipLaunchKernelGGL(ups_reduce_kernel, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, st, part, n_seg, n, upsilon);
    e = hipGetLastError();
  }
  // the host arrays must outlive their asynchronous copies
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const hipError_t ef = hipFreeAsync(ws, st);
  if (e == hipSuccess) e = ef;
  return e == hipSuccess ? RM_OK : pp_hip(fn, e);
}

int rm_group_collision_strengths(const double *omega, int64_t M,
                                 int32_t n_target, const int32_t *group,
                                 int32_t n_group, double *out, void *stream) {
  const char *fn = "rm_group_collision_strengths";
  if (M < 0 || n_target < 1 || n_group < 1)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": M < 0, n_target < 1 or n_group < 1");
  if (!group) return pp_fail(RM_ERR_ARG, std::string(fn) + ": null group");
  for (int t = 0; t < n_target; ++t)
    if (group[t] < 0 || group[t] >= n_group)
      return pp_fail(RM_ERR_ARG, std::string(fn) + ": group index out of range");
  if (M == 0) return RM_OK;
  if (!omega || !out) return pp_fail(RM_ERR_ARG, std::string(fn) + ": null pointer");
  const int64_t P = (int64_t)n_target * (n_target + 1) / 2;
  const int64_t Pg = (int64_t)n_group * (n_group + 1) / 2;
  if (P > 0x7fffffff || Pg > 0x7fffffff)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": too many levels");
  // column lists, grouped by target column
  std::vector<int32_t> cnt(Pg + 1, 0), tgt(P);
  for (int t = 0, p = 0; t < n_target; ++t)
    for (int u = t; u < n_target; ++u, ++p) {
      const int a = std::min(group[t], group[u]), b = std::max(group[t], group[u]);
      tgt[p] = (int32_t)((int64_t)a * n_group - (int64_t)a * (a - 1) / 2 + (b - a));
      ++cnt[tgt[p] + 1];
    }
  std::vector<int32_t> tab(Pg + 1 + P);
  for (int64_t q = 0; q < Pg; ++q) cnt[q + 1] += cnt[q];
  std::copy(cnt.begin(), cnt.end(), tab.begin());
  {
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t p = 0; p < P; ++p) tab[Pg + 1 + pos[tgt[p]]++] = (int32_t)p;
  }
  hipStream_t st = (hipStream_t)stream;
  int32_t *d_tab = nullptr;
  hipError_t e = hipMallocAsync((void **)&d_tab, tab.size() * sizeof(int32_t), st);
  if (e != hipSuccess) return pp_hip(fn, e);
  e = hipMemcpyAsync(d_tab, tab.data(), tab.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    const unsigned grid = (unsigned)std::min<int64_t>(M, 65536);
    hipLaunchKernelGGL(group_kernel, dim3(grid), dim3(256), 0, st, omega, M, P,
                       d_tab, d_tab + Pg + 1, Pg, out);
    e = hipGetLastError();
  }
  // the host table must outlive its asynchronous copy
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const hipError_t ef = hipFreeAsync(d_tab, st);
  if (e == hipSuccess) e = ef;
  return e == hipSuccess ? RM_OK : pp_hip(fn, e);
}

}  // extern "C"
