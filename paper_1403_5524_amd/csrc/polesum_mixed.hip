// Mixed-precision pole sum (paper Sec. 6, Eq. 1-2) with an FP64 near-pole
// correction.
//
//   R_ij(E) = (1/2a) [ sum_{k far} w_ik w_jk d_k  +  sum_{k near} w_ik w_jk d_k ]
//
// with d_k = 1/(E_k - E) formed in FP64 and only then rounded, and "near"
// meaning |E_k - E| < delta (a contiguous index range of the sorted poles).
// The far sum runs on the matrix cores with FP32 accumulation, either
//   * FP32: v_mfma_f32_16x16x4f32 on FP32 W and FP32 d_k w_ik, or
//   * split BF16: x = d_k w_ik and W are each written as hi + lo in BF16 and
//     x W^T ~ xh Wh^T + xh Wl^T + xl Wh^T (v_mfma_f32_16x16x32_bf16), which
//     keeps about 16 significant bits per product;
// the near sum, where d_k is large and FP32 would lose the cancellation in
// E_k - E, is added in FP64 in the epilogue.
//
// Work decomposition: a workgroup owns one 16-row block I of R, a run of up
// to 16 column blocks J >= I (upper triangle), and 8 energies (2 per wave).
// The B operand tiles (W rows of the J blocks) are staged in LDS per chunk of
// 32 poles and shared by all 8 energies; each wave forms its energies'
// scaled A fragments once per chunk and reuses them across all J blocks.
#include "rm_internal.h"

namespace rmx {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int MX_KC = 32;       // poles per chunk
constexpr int MX_JMAX = 16;     // column blocks per workgroup
constexpr int MX_EW = 2;        // energies per wave
constexpr int MX_EG = 8;        // energies per workgroup
constexpr int MX_BPAD = 8;      // LDS row padding (elements) against conflicts

struct MixedArgs {
  const float *W32c;       // [n_pad][nh_pad] channel-major FP32
  const uint16_t *Whc;     // [n_pad][nh_pad] channel-major BF16 hi
  const uint16_t *Wlc;     // [n_pad][nh_pad] channel-major BF16 lo
  const double *Wt;        // [nh_pad][n_pad] pole-major FP64 (near poles)
  const double *Ep;        // [nh_pad]
  const double *E;         // [m]
  double *R;
  int64_t r_estride;
  int r_ld;
  int n, n_pad, nh, nh_pad, m;
  int nblk;                // n_pad / 16
  int njg;                 // column-block groups per row block
  double delta;
  double scale;
};

__device__ inline void decode_rowpanel(int bid, int nblk, int njg, int &IB,
                                       int &JB0, int &grp) {
  // blocks enumerate (IB, JG) pairs with JG covering [IB, nblk) in runs of
  // MX_JMAX; pairs whose run starts past nblk are skipped by the caller.
  const int per = nblk * njg;
  grp = bid / per;
  const int r = bid % per;
  IB = r / njg;
  JB0 = IB + (r % njg) * MX_JMAX;
}

__device__ inline int lower_bound_pole(const double *Ep, int nh, double x) {
  int lo = 0, hi = nh;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (Ep[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <bool BF16>
__global__ __launch_bounds__(256) void polesum_mixed_kernel(MixedArgs p) {
  // B tiles: rows j (MX_JMAX*16), MX_KC poles each (+pad)
  __shared__ float Bf[BF16 ? 1 : MX_JMAX * 16][MX_KC + 1];
  __shared__ unsigned short Bh[BF16 ? MX_JMAX * 16 : 1][MX_KC + MX_BPAD];
  __shared__ unsigned short Bl[BF16 ? MX_JMAX * 16 : 1][MX_KC + MX_BPAD];
  __shared__ float As[16][MX_KC + (BF16 ? 4 : 1)];
  __shared__ float Ds[MX_EG][MX_KC + 4];
  __shared__ int nlo[MX_EG], nhi[MX_EG];

  int IB, JB0, grp;
  decode_rowpanel(blockIdx.x, p.nblk, p.njg, IB, JB0, grp);
  if (JB0 >= p.nblk) return;
  const int nJ = min(MX_JMAX, p.nblk - JB0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int e0 = grp * MX_EG;

  if (tid < MX_EG) {
    const int e = e0 + tid;
    int lo = 0, hi = 0;
    if (e < p.m) {
      const double Ee = p.E[e];
      // superset of the near set; the epilogue applies the exact test
      lo = lower_bound_pole(p.Ep, p.nh, Ee - 2.0 * p.delta);
      hi = lower_bound_pole(p.Ep, p.nh, Ee + 2.0 * p.delta);
    }
    nlo[tid] = lo;
    nhi[tid] = hi;
  }

  f4 acc[MX_EW][MX_JMAX];
#pragma unroll
  for (int e = 0; e < MX_EW; ++e)
#pragma unroll
    for (int b = 0; b < MX_JMAX; ++b) acc[e][b] = f4{0.f, 0.f, 0.f, 0.f};

  const int col = lane & 15, kq = lane >> 4;
  double Eloc = 0.0;
  const int de = tid / MX_KC, dk = tid % MX_KC;  // 256 = 8 energies x 32
  const bool dvalid = (e0 + de) < p.m;
  if (dvalid) Eloc = p.E[e0 + de];

  for (int k0 = 0; k0 < p.nh_pad; k0 += MX_KC) {
    // --- stage B rows (J blocks), A rows (block I) and d
    const int nrows = nJ * 16;
    if (BF16) {
      // 16-byte pieces: each row has MX_KC bf16 = 4 pieces, hi and lo
      for (int q = tid; q < nrows * 4; q += 256) {
        const int r = q >> 2, piece = q & 3;
        const int64_t g = (int64_t)(JB0 * 16 + r) * p.nh_pad + k0 + piece * 8;
        *(uint4 *)&Bh[r][piece * 8] = *(const uint4 *)(p.Whc + g);
        *(uint4 *)&Bl[r][piece * 8] = *(const uint4 *)(p.Wlc + g);
      }
    } else {
      for (int q = tid; q < nrows * 8; q += 256) {
        const int r = q >> 3, piece = q & 7;
        const int64_t g = (int64_t)(JB0 * 16 + r) * p.nh_pad + k0 + piece * 4;
        const float4 v = *(const float4 *)(p.W32c + g);
        Bf[r][piece * 4 + 0] = v.x;
        Bf[r][piece * 4 + 1] = v.y;
        Bf[r][piece * 4 + 2] = v.z;
        Bf[r][piece * 4 + 3] = v.w;
      }
    }
    if (tid < 16 * 8) {
      const int r = tid >> 3, piece = tid & 7;
      const int64_t g = (int64_t)(IB * 16 + r) * p.nh_pad + k0 + piece * 4;
      const float4 v = *(const float4 *)(p.W32c + g);
      As[r][piece * 4 + 0] = v.x;
      As[r][piece * 4 + 1] = v.y;
      As[r][piece * 4 + 2] = v.z;
      As[r][piece * 4 + 3] = v.w;
    }
    {
      float dv = 0.f;
      if (dvalid) {
        const double diff = p.Ep[k0 + dk] - Eloc;   // FP64 subtraction
        if (!(fabs(diff) < p.delta)) dv = (float)(1.0 / diff);
      }
      Ds[de][dk] = dv;
    }
    __syncthreads();

    if (BF16) {
      // lane: row i = col of block I, poles 8*kq .. 8*kq+7
      bf8 xh[MX_EW], xl[MX_EW];
#pragma unroll
      for (int e = 0; e < MX_EW; ++e) {
        const int el = wave * MX_EW + e;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float x = As[col][8 * kq + t] * Ds[el][8 * kq + t];
          const __bf16 h = (__bf16)x;
          xh[e][t] = h;
          xl[e][t] = (__bf16)(x - (float)h);
        }
      }
#pragma unroll
      for (int b = 0; b < MX_JMAX; ++b) {
        if (b < nJ) {
          const int r = b * 16 + col;
          const bf8 bh = *(const bf8 *)&Bh[r][8 * kq];
          const bf8 bl = *(const bf8 *)&Bl[r][8 * kq];
#pragma unroll
          for (int e = 0; e < MX_EW; ++e) {
            f4 c = acc[e][b];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[e], bh, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[e], bl, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[e], bh, c, 0, 0, 0);
            acc[e][b] = c;
          }
        }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < MX_KC; kk += 4) {
        const int kr = kk + kq;
        float xa[MX_EW];
#pragma unroll
        for (int e = 0; e < MX_EW; ++e)
          xa[e] = As[col][kr] * Ds[wave * MX_EW + e][kr];
#pragma unroll
        for (int b = 0; b < MX_JMAX; ++b) {
          if (b < nJ) {
            const float bv = Bf[b * 16 + col][kr];
#pragma unroll
            for (int e = 0; e < MX_EW; ++e)
              acc[e][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                  xa[e], bv, acc[e][b], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // --- epilogue: FP64 near-pole correction and store (both triangles)
#pragma unroll
  for (int e = 0; e < MX_EW; ++e) {
    const int el = wave * MX_EW + e;
    const int eg = e0 + el;
    if (eg >= p.m) continue;
    const double Ee = p.E[eg];
    const int klo = nlo[el], khi = nhi[el];
    double *Re = p.R + (int64_t)eg * p.r_estride;
#pragma unroll
    for (int b = 0; b < MX_JMAX; ++b) {
      if (b >= nJ) continue;
      const int JB = JB0 + b;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = IB * 16 + 4 * kq + r;
        const int gj = JB * 16 + col;
        if (gi >= p.n || gj >= p.n) continue;
        double v = (double)acc[e][b][r];
        for (int k = klo; k < khi; ++k) {
          const double diff = p.Ep[k] - Ee;
          if (!(fabs(diff) < p.delta)) continue;  // same test as the d_k staging
          v += p.Wt[(int64_t)k * p.n_pad + gi] * p.Wt[(int64_t)k * p.n_pad + gj] / diff;
        }
        v *= p.scale;
        Re[(int64_t)gi * p.r_ld + gj] = v;
        if (JB != IB) Re[(int64_t)gj * p.r_ld + gi] = v;
      }
    }
  }
}

hipError_t launch_polesum_mixed(const Sym &s, int prec, double delta,
                                const double *E, int64_t m, double *R,
                                int64_t r_estride, int r_ld, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  MixedArgs p;
  p.W32c = s.W32c;
  p.Whc = s.Whc;
  p.Wlc = s.Wlc;
  p.Wt = s.Wt;
  p.Ep = s.E_pole;
  p.E = E;
  p.R = R;
  p.r_estride = r_estride;
  p.r_ld = r_ld;
  p.n = s.n;
  p.n_pad = s.n_pad;
  p.nh = s.nh;
  p.nh_pad = s.nh_pad;
  p.m = (int)m;
  p.nblk = s.n_pad / 16;
  p.njg = (p.nblk + MX_JMAX - 1) / MX_JMAX;
  p.delta = delta;
  p.scale = 1.0 / (2.0 * s.a);
  const int64_t groups = (m + MX_EG - 1) / MX_EG;
  const int64_t blocks = groups * p.nblk * p.njg;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (prec == RM_PREC_BF16X3)
    hipLaunchKernelGGL(polesum_mixed_kernel<true>, dim3((unsigned)blocks),
                       dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(polesum_mixed_kernel<false>, dim3((unsigned)blocks),
                       dim3(256), 0, st, p);
  return hipGetLastError();
}

}  // namespace rmx
