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
// Omega~ = G Omega, each row of G divided by its sum at the end; it runs on
// the FP64 matrix cores.  A workgroup owns 64 outputs and 256 transitions,
// walks the band of mesh rows its outputs reach in stages of 16, forms those
// rows' weights in LDS (each exp once per workgroup, its row sum kept on the
// way) beside the staged Omega rows, and every wave applies its 16 outputs'
// weights with 16x16x4 MFMAs.  Up to 128 transitions per workgroup keep it
// at 48 KB of LDS and at most 168 registers per lane, so three workgroups
// share a CU and one's staging and barrier overlap the others' MFMAs.  Upsilon and the grouping are single passes over Omega
// (HBM-bound).
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
constexpr int CV_BP = 128;       // transitions per workgroup, at most
constexpr int CV_NB = CV_BP / 16;
constexpr int CV_KC = 16;        // mesh rows per stage

constexpr int CV_OPAD = 16;      // Omega row padding: the four rows an MFMA
                                 // operand spans fall on different banks

struct CvSmem {  // 53 KB: three workgroups per CU
  double O[2][CV_KC][CV_BP + CV_OPAD];
  double W[2][CV_KC][CV_BM];
};

// exp(y) for -745 < y <= 0 (the Gaussian weights): Cody-Waite reduction
// y = n ln2 + t with ln2 split in two (the high part has enough trailing
// zeros that n ln2_hi is exact), exp(t) from its Taylor series to t^13
// (truncation below 5e-18 for |t| <= ln2 / 2), then scaling by 2^n.
__device__ inline double cv_exp(double y) {
  y = fmax(y, -740.0);
  const double n = rint(y * 1.4426950408889634);
  const double t = fma(-n, 1.9082149292705877e-10, fma(-n, 6.93147180369123816490e-01, y));
  double q = 1.0 / 6227020800.0;  // 1/13!
  q = fma(q, t, 1.0 / 479001600.0);
  q = fma(q, t, 1.0 / 39916800.0);
  q = fma(q, t, 1.0 / 3628800.0);
  q = fma(q, t, 1.0 / 362880.0);
  q = fma(q, t, 1.0 / 40320.0);
  q = fma(q, t, 1.0 / 5040.0);
  q = fma(q, t, 1.0 / 720.0);
  q = fma(q, t, 1.0 / 120.0);
  q = fma(q, t, 1.0 / 24.0);
  q = fma(q, t, 1.0 / 6.0);
  q = fma(q, t, 0.5);
  q = fma(q, t, 1.0);
  q = fma(q, t, 1.0);
  return ldexp(q, (int)n);
}

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

// Trapezoid weights dE and each output's window [lo, hi).
__global__ void conv_window_kernel(const double *__restrict__ E, int64_t m,
                                   double s, double *dE, int64_t *lo,
                                   int64_t *hi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double Ei = E[i];
  double w = 0.0;
  if (i > 0) w += 0.5 * (Ei - E[i - 1]);
  if (i + 1 < m) w += 0.5 * (E[i + 1] - Ei);
  dE[i] = w;
  lo[i] = pp_first_ge(E, m, Ei - CV_CUT * s);
  hi[i] = pp_first_gt(E, m, Ei + CV_CUT * s);
}

// NB column blocks of 16 per workgroup (the column tiles split the
// transitions evenly, the last one may be narrower), so the MFMA loop has no
// branches.
template <int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3)))
void conv_apply_kernel(const double *__restrict__ E,
                       const double *__restrict__ dE, int64_t m,
                       const double *__restrict__ in, int64_t P, int64_t pbase,
                       double r, const int64_t *__restrict__ lo,
                       const int64_t *__restrict__ hi,
                       double *__restrict__ out, int n_tiles) {
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
  const int64_t p0 = pbase + (int64_t)blockIdx.y * (16 * NB);
  const int64_t jlo = lo[i0], jhi = hi[ilast];

  // this wave's 16 outputs and the rows they reach
  const int64_t wi0 = i0 + 16 * wave;
  const bool wact = wi0 <= ilast;
  const int64_t wlo = wact ? lo[wi0] : 0;
  const int64_t whi = wact ? hi[min<int64_t>(wi0 + 15, ilast)] : 0;

  // weight staging: output i0 + lane, stage rows wave + 4 u (wave-uniform,
  // so E and dE of a row come through the scalar cache)
  const int64_t gi = i0 + lane;
  const bool iv = gi <= ilast;
  const double Ei = E[min(gi, ilast)];
  const int64_t ilo = iv ? lo[gi] : 0, ihi = iv ? hi[gi] : 0;
  double gsum = 0.0;  // this thread's share of sum_j g_ij
  // Omega staging: column p0 + (tid % 128), rows tid / 128 + 2 k of a stage.
  // Loads are clamped into the band and the array: a clamped value meets a
  // zero weight or feeds a column that is never stored.
  const int sc = tid & (CV_BP - 1);
  const int sr = __builtin_amdgcn_readfirstlane(tid >> 7);  // wave-uniform
  const int64_t col_off = min(p0 + sc, P - 1);

  double rO[CV_KC / 2], rW[4];
  // one quarter of a stage: Omega rows sr + 2 k for k = 2 h, 2 h + 1 and the
  // weight of row wave + 4 h
  auto fetch_part = [&](int64_t j0, int h) {
#pragma unroll
    for (int k = 2 * h; k < 2 * h + 2; ++k) {
      // row base in scalar registers, column offset per lane
      const double *row = in + min(j0 + sr + 2 * k, jhi - 1) * P;
      rO[k] = row[col_off];
    }
    const int64_t j = j0 + wave + 4 * h;
    const int64_t jc = min(j, m - 1);
    const double x = E[jc] - Ei;
    const double w = cv_exp(-r * x * x) * dE[jc];
    rW[h] = (j >= ilo && j < ihi) ? w : 0.0;
    gsum += rW[h];
  };
  auto stage = [&](int b) {
#pragma unroll
    for (int k = 0; k < CV_KC / 2; ++k) sm.O[b][sr + 2 * k][sc] = rO[k];
#pragma unroll
    for (int u = 0; u < 4; ++u) sm.W[b][wave + 4 * u][lane] = rW[u];
  };

  d4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = d4{0.0, 0.0, 0.0, 0.0};
  const int kq = lane >> 4;
  const int col = lane & 15;

#pragma unroll
  for (int h = 0; h < 4; ++h) fetch_part(jlo, h);
  stage(0);
  if (jlo + CV_KC < jhi) {
#pragma unroll
    for (int h = 0; h < 4; ++h) fetch_part(jlo + CV_KC, h);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t j0 = jlo; j0 < jhi; j0 += CV_KC, buf ^= 1) {
    // the next stage, fetched during the previous one, goes to the other
    // buffer (free since the last barrier); the one after it is fetched in
    // four parts between this stage's MFMA steps
    const bool more = j0 + CV_KC < jhi;
    const bool more2 = j0 + 2 * CV_KC < jhi;
    if (more) stage(buf ^ 1);
    if (wact && j0 < whi && j0 + CV_KC > wlo) {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int kk = 4 * h;
        const double a = sm.W[buf][kk + kq][16 * wave + col];
        double bv[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) bv[b] = sm.O[buf][kk + kq][16 * b + col];
#pragma unroll
        for (int b = 0; b < NB; ++b)
          acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[b], acc[b], 0, 0, 0);
        if (more2) fetch_part(j0 + 2 * CV_KC, h);
      }
    } else if (more2) {
#pragma unroll
      for (int h = 0; h < 4; ++h) fetch_part(j0 + 2 * CV_KC, h);
    }
    __syncthreads();
  }
  // row sums: the four staging threads of each output add their shares
  // (the weight buffers are free after the last barrier)
  double(*s_sum)[CV_BM] = sm.W[0];
  s_sum[wave][lane] = gsum;
  __syncthreads();

  // FP64 16x16x4 result: lane holds row kq + 4 q, column col of its block
  if (wact) {
    double inv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int li = 16 * wave + kq + 4 * q;
      inv[q] = 1.0 / (((s_sum[0][li] + s_sum[1][li]) + s_sum[2][li]) + s_sum[3][li]);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int64_t p = p0 + 16 * b + col;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t i = wi0 + kq + 4 * q;
        if (i <= ilast && p < P) out[i * P + p] = acc[b][q] * inv[q];
      }
    }
  }
}

template <int NB>
static void launch_conv_apply(dim3 grid, hipStream_t st, const double *E,
                              const double *dE, int64_t M, const double *in,
                              int64_t P, int64_t pbase, double r,
                              const int64_t *lo, const int64_t *hi,
                              double *out, int n_tiles) {
  hipLaunchKernelGGL(conv_apply_kernel<NB>, grid, dim3(256), 0, st, E, dE, M,
                     in, P, pbase, r, lo, hi, out, n_tiles);
}

typedef void (*ConvLaunch)(dim3, hipStream_t, const double *, const double *,
                           int64_t, const double *, int64_t, int64_t, double,
                           const int64_t *, const int64_t *, double *, int);
static const ConvLaunch kConvLaunch[CV_NB + 1] = {
    nullptr,              launch_conv_apply<1>, launch_conv_apply<2>,
    launch_conv_apply<3>, launch_conv_apply<4>, launch_conv_apply<5>,
    launch_conv_apply<6>, launch_conv_apply<7>, launch_conv_apply<8>};

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

constexpr int UP_T = 8;    // temperatures per pass over Omega
constexpr int UP_W = 8;    // mesh segments (waves) per workgroup
constexpr int UP_R = 8;    // mesh rows per block; the next block is in flight

__device__ inline int64_t wave_min64(int64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int64_t o = __shfl_xor(v, off);
    v = min(v, o);
  }
  return v;
}

__device__ inline int64_t uniform64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline double lane_value(double v, int l) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One transition per lane and one mesh segment per wave; the 8 waves of a
// workgroup add their segments in LDS and write one partial sum per pass:
// part [gridDim.y][P][nT].  y_q = exp(-eps/kT_q) / kT_q starts exact at each
// lane's first row and then follows the product of the per-interval factors
// f.  A block of 8 rows loads its factors (lane 8 k + q: row k, temperature
// q) and mesh energies E[ib - 1 .. ib + 8] as one vector each, parks them in
// the wave's LDS slot and reads them back as broadcasts.
__global__ __launch_bounds__(512) void ups_part_kernel(
    const double *__restrict__ E, int64_t m, const double *__restrict__ om,
    int n_target, int64_t P, const double *__restrict__ e_level,
    const double *__restrict__ kT, int nT, const double *__restrict__ f,
    int64_t seg_len, double *__restrict__ part) {
  __shared__ double red[UP_W][UP_T][64];
  __shared__ double blk[UP_W][UP_R * UP_T + 16];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t seg = (int64_t)blockIdx.y * UP_W + wave;
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const bool pv = p < P;
  const int64_t pc = pv ? p : P - 1;
  // level pair (t, u), t <= u, of packed index p
  int t = 0;
  int64_t rem = pc;
  while (rem >= n_target - t) {
    rem -= n_target - t;
    ++t;
  }
  const int u = t + (int)rem;
  const double e = fmax(e_level[t], e_level[u]);
  const int64_t i0 = pp_first_gt(E, m, e);  // first point above e
  const int64_t s_lo = min(m, seg * seg_len);
  const int64_t s_hi = min(m, s_lo + seg_len);
  const int64_t first = pv ? max(i0, s_lo) : m;
  const int64_t istart = uniform64(wave_min64(first));
  const int64_t mlast = m > 0 ? m - 1 : 0;
  double *slot = blk[wave];

  for (int t0 = 0; t0 < nT; t0 += UP_T) {
    const int nt = min(UP_T, nT - t0);
    double T[UP_T], iT[UP_T], acc[UP_T], y[UP_T];
#pragma unroll
    for (int q = 0; q < UP_T; ++q) {
      T[q] = kT[t0 + min(q, nt - 1)];
      iT[q] = 1.0 / T[q];
      acc[q] = 0.0;
      y[q] = 0.0;
    }
    // block loads, clamped into the arrays (masked when used)
    const int fq = min(lane & 7, nt - 1);
    auto load = [&](int64_t ib, double *v, double &fv, double &ev) {
#pragma unroll
      for (int k = 0; k < UP_R; ++k) v[k] = om[min(ib + k, mlast) * P + pc];
      fv = f[min(ib + (lane >> 3), mlast) * nT + t0 + fq];
      const int64_t ie = min(ib - 1 + lane, mlast);
      ev = E[ie < 0 ? 0 : ie];
    };
    double va[UP_R], fa, ea;
    if (istart < s_hi) load(istart, va, fa, ea);
    for (int64_t ib = istart; ib < s_hi; ib += UP_R) {
      double vn[UP_R], fn, en;
      load(ib + UP_R, vn, fn, en);
      wave_lds_sync();  // the previous block's reads are done
      slot[lane] = fa;
      if (lane < UP_R + 2) slot[UP_R * UP_T + lane] = ea;
      wave_lds_sync();
#pragma unroll
      for (int k = 0; k < UP_R; ++k) {
        const int64_t i = ib + k;
        const bool act = i >= first && i < s_hi;
        const double v = act ? va[k] : 0.0;
        const double Em = slot[UP_R * UP_T + k];
        const double Ec = slot[UP_R * UP_T + k + 1];
        const double Ep = slot[UP_R * UP_T + k + 2];
        const double wr = i + 1 < m ? 0.5 * (Ep - Ec) : 0.0;
        const double wl = (act && i > i0) ? 0.5 * (Ec - Em) : 0.0;
        if (act && i == first) {
#pragma unroll
          for (int q = 0; q < UP_T; ++q) {
            const double x = exp(-(Ec - e) * iT[q]);
            y[q] = x * iT[q];
            if (i == i0) acc[q] = v * (1.0 - x);  // Omega constant from threshold
          }
        } else {
#pragma unroll
          for (int q = 0; q < UP_T; ++q) y[q] *= slot[UP_T * k + q];
        }
        const double vw = v * (wl + wr);
#pragma unroll
        for (int q = 0; q < UP_T; ++q) acc[q] = fma(vw, y[q], acc[q]);
      }
#pragma unroll
      for (int k = 0; k < UP_R; ++k) va[k] = vn[k];
      fa = fn;
      ea = en;
    }
#pragma unroll
    for (int q = 0; q < UP_T; ++q) red[wave][q][lane] = acc[q];
    __syncthreads();
    if (tid < UP_T * 64) {
      const int q = tid >> 6, l = tid & 63;
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < UP_W; ++w) s += red[w][q][l];
      const int64_t pp = (int64_t)blockIdx.x * 64 + l;
      if (pp < P && q < nt) part[((int64_t)blockIdx.y * P + pp) * nT + t0 + q] = s;
    }
    __syncthreads();
  }
}

__global__ void ups_reduce_kernel(const double *__restrict__ part,
                                  int64_t n_part, int64_t n, double *ups) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double s = 0.0;
#pragma unroll 8
  for (int64_t g = 0; g < n_part; ++g) s += part[g * n + q];
  ups[q] = s;
}

// s + base[cols[k0]] + ... + base[cols[k1 - 1]], added in that order; the
// indices are fetched 8 at a time so their loads overlap.
__device__ inline double gather_sum(const double *base,
                                    const int32_t *__restrict__ cols, int k0,
                                    int k1, double s) {
  int k = k0;
  for (; k + 8 <= k1; k += 8) {
    int c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = cols[k + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += base[c[u]];
  }
  for (; k < k1; ++k) s += base[cols[k]];
  return s;
}

constexpr int GR_LDS = 4096;  // doubles of Omega rows staged per workgroup

// out [m][Pg]: each group pair q sums its level-pair columns
// cols[off[q] .. off[q + 1]).  A workgroup copies `rows` whole rows of Omega
// into LDS with coalesced loads, then forms their outputs from LDS.
__global__ __launch_bounds__(256) void group_lds_kernel(
    const double *__restrict__ om, int64_t m, int64_t P, int rows,
    const int32_t *__restrict__ off, const int32_t *__restrict__ cols,
    int64_t Pg, double *__restrict__ out) {
  __shared__ double buf[GR_LDS];
  const int64_t i0 = (int64_t)blockIdx.x * rows;
  const int nr = (int)min<int64_t>(rows, m - i0);
  const double *src = om + i0 * P;
  for (int64_t k = threadIdx.x; k < nr * P; k += 256) buf[k] = src[k];
  __syncthreads();
  for (int64_t o = threadIdx.x; o < nr * Pg; o += 256) {
    const int64_t r = o / Pg, q = o % Pg;
    const double *row = buf + r * P;
    double s = 0.0;
    s = gather_sum(row, cols, off[q], off[q + 1], s);
    out[i0 * Pg + o] = s;
  }
}

constexpr int GR_ACC = 4096;  // group pairs accumulated in LDS

// Rows longer than GR_LDS: one row at a time in chunks of GR_LDS columns;
// chunk c's columns of group pair q are cols[off[c Pg + q] ..
// off[c Pg + q + 1]) (offsets inside the chunk, ascending), added to an LDS
// accumulator owned by one thread, so every sum runs in ascending column
// order.
__global__ __launch_bounds__(256) void group_chunks_kernel(
    const double *__restrict__ om, int64_t m, int64_t P, int n_ch,
    const int32_t *__restrict__ off, const int32_t *__restrict__ cols,
    int64_t Pg, double *__restrict__ out) {
  __shared__ double buf[GR_LDS];
  __shared__ double acc[GR_ACC];
  const int tid = threadIdx.x;
  for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
    for (int64_t q = tid; q < Pg; q += 256) acc[q] = 0.0;
    const double *row = om + i * P;
    for (int c = 0; c < n_ch; ++c) {
      const int64_t base = (int64_t)c * GR_LDS;
      const int len = (int)min<int64_t>(GR_LDS, P - base);
      __syncthreads();  // the previous chunk has been consumed
      double v[GR_LDS / 256];
#pragma unroll
      for (int u = 0; u < GR_LDS / 256; ++u) {
        const int k = tid + 256 * u;
        v[u] = row[base + min(k, len - 1)];
      }
#pragma unroll
      for (int u = 0; u < GR_LDS / 256; ++u) buf[tid + 256 * u] = v[u];
      __syncthreads();
      for (int64_t q = tid; q < Pg; q += 256) {
        double s = acc[q];
        const int64_t o = (int64_t)c * Pg + q;
        s = gather_sum(buf, cols, off[o], off[o + 1], s);
        acc[q] = s;
      }
    }
    for (int64_t q = tid; q < Pg; q += 256) out[i * Pg + q] = acc[q];
  }
}

// the same from global memory, for rows too long for LDS
__global__ void group_kernel(const double *__restrict__ om, int64_t m,
                             int64_t P, const int32_t *__restrict__ off,
                             const int32_t *__restrict__ cols, int64_t Pg,
                             double *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * Pg) return;
  const int64_t i = idx / Pg, q = idx % Pg;
  const double *row = om + i * P;
  double s = 0.0;
  s = gather_sum(row, cols, off[q], off[q + 1], s);
  out[idx] = s;
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
  if (n_tiles > (int64_t)1 << 30 || (P + 15) / 16 > 65535)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": M or P too large");
  const double s = fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  const double r = 0.5 / (s * s);
  char *ws = nullptr;
  const size_t bytes = (size_t)M * (sizeof(double) + 2 * sizeof(int64_t));
  hipError_t e = hipMallocAsync((void **)&ws, bytes, st);
  if (e != hipSuccess) return pp_hip(fn, e);
  double *dE = (double *)ws;
  int64_t *lo = (int64_t *)(dE + M);
  int64_t *hi = lo + M;
  hipLaunchKernelGGL(conv_window_kernel, dim3((unsigned)((M + 255) / 256)),
                     dim3(256), 0, st, E, M, s, dE, lo, hi);
  e = hipGetLastError();
  if (e == hipSuccess) {
    // column tiles of nb blocks of 16 (at most 8), as even as they come;
    // the last one takes what is left
    const unsigned gx = (unsigned)(8 * ((n_tiles + 7) / 8));
    const int64_t blocks = (P + 15) / 16;
    const int64_t n_ct = (blocks + CV_NB - 1) / CV_NB;
    const int nb = (int)((blocks + n_ct - 1) / n_ct);
    const int64_t full = blocks / nb;
    const int nb_last = (int)(blocks - full * nb);
    ProfileScope prof(4, st);
    if (full > 0)
      kConvLaunch[nb](dim3(gx, (unsigned)full), st, E, dE, M, omega_in, P, 0,
                      r, lo, hi, omega_out, (int)n_tiles);
    if (nb_last > 0)
      kConvLaunch[nb_last](dim3(gx, 1), st, E, dE, M, omega_in, P,
                           full * nb * 16, r, lo, hi, omega_out, (int)n_tiles);
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
  // about 4096 waves, no segment shorter than 64 rows
  int64_t n_seg = std::max<int64_t>(1, std::min<int64_t>((4096 + n_col - 1) / n_col,
                                                         (M + 63) / 64));
  const int64_t seg_len = std::max<int64_t>(1, (M + n_seg - 1) / n_seg);
  n_seg = std::max<int64_t>(1, (M + seg_len - 1) / seg_len);
  const int64_t n_part = (n_seg + UP_W - 1) / UP_W;
  if (n_col > 0x7fffffff || n_part > 65535)
    return pp_fail(RM_ERR_ARG, std::string(fn) + ": M or n_target too large");
  const size_t bytes = sizeof(double) *
      ((size_t)n_target + nT + std::max<size_t>(1, (size_t)M * nT) +
       (size_t)n_part * P * nT);
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
    ProfileScope prof(5, st);
    hipLaunchKernelGGL(ups_part_kernel, dim3((unsigned)n_col, (unsigned)n_part),
                       dim3(64 * UP_W), 0, st, E, M, omega, n_target, P,
                       d_lev, d_kT, nT, f, seg_len, part);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int64_t n = P * nT;
    hipLaunchKernelGGL(ups_reduce_kernel, dim3((unsigned)((n + 255) / 256)),
                       dim3(256), 0, st, part, n_part, n, upsilon);
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
  // column lists per (chunk, group pair), columns ascending within each
  // (one chunk holding every column when a row fits in LDS)
  const bool chunked = P > GR_LDS && Pg <= GR_ACC;
  const bool in_lds = P <= GR_LDS || chunked;
  const int64_t n_ch = chunked ? (P + GR_LDS - 1) / GR_LDS : 1;
  const int64_t n_key = n_ch * Pg;
  std::vector<int32_t> cnt(n_key + 1, 0), key(P);
  for (int t = 0, p = 0; t < n_target; ++t)
    for (int u = t; u < n_target; ++u, ++p) {
      const int a = std::min(group[t], group[u]), b = std::max(group[t], group[u]);
      const int64_t q = (int64_t)a * n_group - (int64_t)a * (a - 1) / 2 + (b - a);
      key[p] = (int32_t)((chunked ? p / GR_LDS : 0) * Pg + q);
      ++cnt[key[p] + 1];
    }
  std::vector<int32_t> tab(n_key + 1 + P);
  for (int64_t q = 0; q < n_key; ++q) cnt[q + 1] += cnt[q];
  std::copy(cnt.begin(), cnt.end(), tab.begin());
  {
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t p = 0; p < P; ++p)
      tab[n_key + 1 + pos[key[p]]++] = (int32_t)(chunked ? p % GR_LDS : p);
  }
  hipStream_t st = (hipStream_t)stream;
  int32_t *d_tab = nullptr;
  hipError_t e = hipMallocAsync((void **)&d_tab, tab.size() * sizeof(int32_t), st);
  if (e != hipSuccess) return pp_hip(fn, e);
  e = hipMemcpyAsync(d_tab, tab.data(), tab.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    ProfileScope prof(6, st);
    const int32_t *d_off = d_tab, *d_cols = d_tab + n_key + 1;
    if (P <= GR_LDS) {
      const int rows = (int)std::min<int64_t>(64, GR_LDS / P);
      hipLaunchKernelGGL(group_lds_kernel, dim3((unsigned)((M + rows - 1) / rows)),
                         dim3(256), 0, st, omega, M, P, rows, d_off, d_cols,
                         Pg, out);
    } else if (in_lds) {
      hipLaunchKernelGGL(group_chunks_kernel,
                         dim3((unsigned)std::min<int64_t>(M, 4096)), dim3(256),
                         0, st, omega, M, P, (int)n_ch, d_off, d_cols, Pg, out);
    } else {
      hipLaunchKernelGGL(group_kernel, dim3((unsigned)((M * Pg + 255) / 256)),
                         dim3(256), 0, st, omega, M, P, d_off, d_cols, Pg, out);
    }
    e = hipGetLastError();
  }
  // the host table must outlive its asynchronous copy
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const hipError_t ef = hipFreeAsync(d_tab, st);
  if (e == hipSuccess) e = ef;
  return e == hipSuccess ? RM_OK : pp_hip(fn, e);
}

}  // extern "C"
