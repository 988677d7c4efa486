// Pole-sum contraction (paper Sec. 6, Eq. 1-2) on gfx950 matrix cores.
//
// R(E) = (1/2a) W diag(d(E)) W^T with d_k(E) = 1/(E_k - E): per energy a
// symmetric n x n product whose shared operand W (n x N_H) is the same for
// every energy.  One workgroup owns an upper-triangle tile pair (I, J) of
// 32 x 32 outputs and a group of 16 energies; W tiles of 32 poles are staged
// in LDS once and reused by all 16 energies, each wave scaling the A
// fragment by its own d_k(E) before the MFMA.  Only tile pairs I <= J are
// computed; the mirror block is written from the same accumulators.
#include "rm_internal.h"

namespace rmx {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int PS_T = 32;    // output tile edge
constexpr int PS_KC = 32;   // poles per LDS stage
constexpr int PS_EW = 4;    // energies per wave
constexpr int PS_EG = 16;   // energies per workgroup (4 waves)

struct PoleSumF64Args {
  const double *Wt;     // [nh_pad][n_pad]
  const double *Ep;     // [nh_pad]
  const double *E;      // [m]
  double *R;
  int64_t r_estride;
  int r_ld;
  int n, n_pad, nh_pad, m;
  int ntile, npairs;
  double scale;
};

__device__ inline void pair_to_tiles(int pair, int ntile, int &I, int &J) {
  int i = 0, rem = pair;
  while (rem >= ntile - i) {
    rem -= ntile - i;
    ++i;
  }
  I = i;
  J = i + rem;
}

__global__ __launch_bounds__(256) void polesum_f64_kernel(PoleSumF64Args p) {
  __shared__ double As[PS_KC][PS_T];
  __shared__ double Bs[PS_KC][PS_T];
  __shared__ double Ds[PS_EG][PS_KC];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int pair = blockIdx.x % p.npairs;
  const int group = blockIdx.x / p.npairs;
  int I, J;
  pair_to_tiles(pair, p.ntile, I, J);
  const int e0 = group * PS_EG;
  const bool diag = (I == J);

  // staging roles: 8 threads per pole row, 4 doubles each
  const int ld_k = tid >> 3;          // 0..31
  const int ld_c = (tid & 7) * 4;     // 0..28
  const double *wa = p.Wt + (int64_t)ld_k * p.n_pad + I * PS_T + ld_c;
  const double *wb = p.Wt + (int64_t)ld_k * p.n_pad + J * PS_T + ld_c;
  // d roles: 2 values per thread
  double Eloc[2];
  int dk[2], de[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int idx = tid + 256 * u;
    de[u] = idx / PS_KC;
    dk[u] = idx % PS_KC;
    const int e = e0 + de[u];
    Eloc[u] = (e < p.m) ? p.E[e] : 0.0;
  }
  const bool evalid0 = (e0 + de[0]) < p.m, evalid1 = (e0 + de[1]) < p.m;

  d4 acc[PS_EW][2][2];
#pragma unroll
  for (int e = 0; e < PS_EW; ++e)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[e][a][b] = d4{0.0, 0.0, 0.0, 0.0};

  const int col = lane & 15;
  const int kq = lane >> 4;

  // register prefetch of stage 0
  double2 ra0 = *(const double2 *)(wa);
  double2 ra1 = *(const double2 *)(wa + 2);
  double2 rb0 = ra0, rb1 = ra1;
  if (!diag) {
    rb0 = *(const double2 *)(wb);
    rb1 = *(const double2 *)(wb + 2);
  }
  double ep0 = p.Ep[dk[0]], ep1 = p.Ep[dk[1]];

  for (int k0 = 0; k0 < p.nh_pad; k0 += PS_KC) {
    *(double2 *)&As[ld_k][ld_c] = ra0;
    *(double2 *)&As[ld_k][ld_c + 2] = ra1;
    if (!diag) {
      *(double2 *)&Bs[ld_k][ld_c] = rb0;
      *(double2 *)&Bs[ld_k][ld_c + 2] = rb1;
    }
    Ds[de[0]][dk[0]] = evalid0 ? 1.0 / (ep0 - Eloc[0]) : 0.0;
    Ds[de[1]][dk[1]] = evalid1 ? 1.0 / (ep1 - Eloc[1]) : 0.0;
    __syncthreads();
    const int kn = k0 + PS_KC;
    if (kn < p.nh_pad) {
      const int64_t off = (int64_t)kn * p.n_pad;
      ra0 = *(const double2 *)(wa + off);
      ra1 = *(const double2 *)(wa + off + 2);
      if (!diag) {
        rb0 = *(const double2 *)(wb + off);
        rb1 = *(const double2 *)(wb + off + 2);
      }
      ep0 = p.Ep[kn + dk[0]];
      ep1 = p.Ep[kn + dk[1]];
    }
    const double(*Bsel)[PS_T] = diag ? As : Bs;
#pragma unroll
    for (int kk = 0; kk < PS_KC; kk += 4) {
      const int kr = kk + kq;
      const double a0 = As[kr][col];
      const double a1 = As[kr][16 + col];
      const double b0 = Bsel[kr][col];
      const double b1 = Bsel[kr][16 + col];
#pragma unroll
      for (int e = 0; e < PS_EW; ++e) {
        const double dd = Ds[wave * PS_EW + e][kr];
        const double sa0 = a0 * dd, sa1 = a1 * dd;
        acc[e][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa0, b0, acc[e][0][0], 0, 0, 0);
        acc[e][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa0, b1, acc[e][0][1], 0, 0, 0);
        acc[e][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa1, b0, acc[e][1][0], 0, 0, 0);
        acc[e][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa1, b1, acc[e][1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // epilogue: for the FP64 16x16x4 MFMA, lane holds D[i][j] with
  // j = lane % 16 and i = lane / 16 + 4 r (rows interleaved across the four
  // result registers; the FP32/BF16 forms use i = 4 (lane / 16) + r)
#pragma unroll
  for (int e = 0; e < PS_EW; ++e) {
    const int eg = e0 + wave * PS_EW + e;
    if (eg >= p.m) continue;
    double *Re = p.R + (int64_t)eg * p.r_estride;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = I * PS_T + a * 16 + kq + 4 * r;
          const int gj = J * PS_T + b * 16 + col;
          if (gi < p.n && gj < p.n) {
            const double v = acc[e][a][b][r] * p.scale;
            Re[(int64_t)gi * p.r_ld + gj] = v;
            if (!diag) Re[(int64_t)gj * p.r_ld + gi] = v;
          }
        }
  }
}

hipError_t launch_polesum_f64(const Sym &s, const double *E, int64_t m,
                              double *R, int64_t r_estride, int r_ld,
                              hipStream_t st) {
  if (m <= 0) return hipSuccess;
  PoleSumF64Args p;
  p.Wt = s.Wt;
  p.Ep = s.E_pole;
  p.E = E;
  p.R = R;
  p.r_estride = r_estride;
  p.r_ld = r_ld;
  p.n = s.n;
  p.n_pad = s.n_pad;
  p.nh_pad = s.nh_pad;
  p.m = (int)m;
  p.ntile = s.n_pad / PS_T;
  p.npairs = p.ntile * (p.ntile + 1) / 2;
  p.scale = 1.0 / (2.0 * s.a);
  const int64_t groups = (m + PS_EG - 1) / PS_EG;
  const int64_t blocks = groups * p.npairs;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(polesum_f64_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     st, p);
  return hipGetLastError();
}

}  // namespace rmx
