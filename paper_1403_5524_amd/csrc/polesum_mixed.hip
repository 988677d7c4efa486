// Mixed-precision pole sum (paper Sec. 6, Eq. 1-2) in three tiers.
//
//   R_ij(E) = (1/2a) [ sum_{k far} + sum_{k band} + sum_{k near} ] w_ik w_jk d_k
//
// with d_k = 1/(E_k - E) formed in FP64 and only then rounded; "near" means
// |E_k - E| < delta, "band" delta <= |E_k - E| < band (contiguous index
// ranges of the sorted poles), "far" the rest.
// The far sum runs on the matrix cores with FP32 accumulation, either
//   * FP32: v_mfma_f32_16x16x4f32 on FP32 W and FP32 d_k w_ik, or
//   * split BF16: x = d_k w_ik and W are each written as hi + lo in BF16 and
//     x W^T ~ xh Wh^T + xh Wl^T + xl Wh^T (v_mfma_f32_16x16x32_bf16), which
//     keeps about 16 significant bits per product;
// the near sum, where d_k is large and FP32 would lose the cancellation in
// E_k - E, is added in FP64 in the epilogue, and so is the band sum from
// FP32-rounded w_ik, w_jk and d_k (FP64 products and sum): its terms are the
// largest of the rest, and accumulated in FP32 they would set the rounding
// of every term added after them.
//
// Work decomposition: a work item is one 16-row block I of R of one
// symmetry, a run of up to JMAX column blocks J >= I (upper triangle), and
// 4*EW energies (EW per wave).  The B operand tiles (W rows of the J blocks)
// are staged in LDS per chunk of 32 poles and shared by all energies of the
// item; each wave forms its energies' scaled A fragments once per chunk and
// reuses them across all J blocks.  JMAX and EW are the tile variants the
// autotuner chooses between.
#include <algorithm>

#include "rm_internal.h"

namespace rmx {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int MX_KC = 32;       // poles per chunk
constexpr int MX_BPAD = 8;      // LDS row padding (elements) against conflicts

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

template <bool BF16, int JMAX, int EW>
struct MxSmem {
  float Bf[BF16 ? 1 : JMAX * 16][MX_KC + 1];
  unsigned short Bh[BF16 ? JMAX * 16 : 1][MX_KC + MX_BPAD];
  unsigned short Bl[BF16 ? JMAX * 16 : 1][MX_KC + MX_BPAD];
  float As[16][MX_KC + (BF16 ? 4 : 1)];
  float Ds[4 * EW][MX_KC + 4];
  int nlo[4 * EW], nhi[4 * EW];
};

template <bool BF16, int JMAX, int EW>
__device__ void ps_mixed_item(const SymDev &S, int IB, int JB0, int grp,
                              const double *__restrict__ E, int m,
                              double delta, double band,
                              double *__restrict__ Rbase,
                              int64_t estride, int ld,
                              MxSmem<BF16, JMAX, EW> &sm) {
  constexpr int EG = 4 * EW;
  const int nblk = S.n_pad / 16;
  const int nJ = min(JMAX, nblk - JB0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int e0 = grp * EG;
  const int nh_pad = S.nh_pad;

  if (tid < EG) {
    const int e = e0 + tid;
    int lo = 0, hi = 0;
    if (e < m) {
      const double Ee = E[e];
      // superset of the near and band tiers; the epilogue applies the
      // exact tests
      lo = lower_bound_pole(S.E_pole, S.nh, Ee - 2.0 * band);
      hi = lower_bound_pole(S.E_pole, S.nh, Ee + 2.0 * band);
    }
    sm.nlo[tid] = lo;
    sm.nhi[tid] = hi;
  }

  f4 acc[EW][JMAX];
#pragma unroll
  for (int e = 0; e < EW; ++e)
#pragma unroll
    for (int b = 0; b < JMAX; ++b) acc[e][b] = f4{0.f, 0.f, 0.f, 0.f};

  const int col = lane & 15, kq = lane >> 4;
  // d staging: EG energies x 32 poles over 256 threads
  constexpr int DPER = (EG * MX_KC + 255) / 256;

  for (int k0 = 0; k0 < nh_pad; k0 += MX_KC) {
    const int nrows = nJ * 16;
    if (BF16) {
      for (int q = tid; q < nrows * 4; q += 256) {
        const int r = q >> 2, piece = q & 3;
        const int64_t g = (int64_t)(JB0 * 16 + r) * nh_pad + k0 + piece * 8;
        *(uint4 *)&sm.Bh[r][piece * 8] = *(const uint4 *)(S.Whc + g);
        *(uint4 *)&sm.Bl[r][piece * 8] = *(const uint4 *)(S.Wlc + g);
      }
    } else {
      for (int q = tid; q < nrows * 8; q += 256) {
        const int r = q >> 3, piece = q & 7;
        const int64_t g = (int64_t)(JB0 * 16 + r) * nh_pad + k0 + piece * 4;
        const float4 v = *(const float4 *)(S.W32c + g);
        sm.Bf[r][piece * 4 + 0] = v.x;
        sm.Bf[r][piece * 4 + 1] = v.y;
        sm.Bf[r][piece * 4 + 2] = v.z;
        sm.Bf[r][piece * 4 + 3] = v.w;
      }
    }
    if (tid < 16 * 8) {
      const int r = tid >> 3, piece = tid & 7;
      const int64_t g = (int64_t)(IB * 16 + r) * nh_pad + k0 + piece * 4;
      const float4 v = *(const float4 *)(S.W32c + g);
      sm.As[r][piece * 4 + 0] = v.x;
      sm.As[r][piece * 4 + 1] = v.y;
      sm.As[r][piece * 4 + 2] = v.z;
      sm.As[r][piece * 4 + 3] = v.w;
    }
#pragma unroll
    for (int u = 0; u < DPER; ++u) {
      const int q = tid + 256 * u;
      if (q < EG * MX_KC) {
        const int de = q / MX_KC, dk = q % MX_KC;
        float dv = 0.f;
        if (e0 + de < m) {
          const double diff = S.E_pole[k0 + dk] - E[e0 + de];  // FP64
          if (!(fabs(diff) < band)) dv = (float)(1.0 / diff);
        }
        sm.Ds[de][dk] = dv;
      }
    }
    __syncthreads();

    if (BF16) {
      bf8 xh[EW], xl[EW];
#pragma unroll
      for (int e = 0; e < EW; ++e) {
        const int el = wave * EW + e;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const float x = sm.As[col][8 * kq + t] * sm.Ds[el][8 * kq + t];
          const __bf16 h = (__bf16)x;
          xh[e][t] = h;
          xl[e][t] = (__bf16)(x - (float)h);
        }
      }
#pragma unroll
      for (int b = 0; b < JMAX; ++b) {
        if (b < nJ) {
          const int r = b * 16 + col;
          const bf8 bh = *(const bf8 *)&sm.Bh[r][8 * kq];
          const bf8 bl = *(const bf8 *)&sm.Bl[r][8 * kq];
#pragma unroll
          for (int e = 0; e < EW; ++e) {
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
        float xa[EW];
#pragma unroll
        for (int e = 0; e < EW; ++e)
          xa[e] = sm.As[col][kr] * sm.Ds[wave * EW + e][kr];
#pragma unroll
        for (int b = 0; b < JMAX; ++b) {
          if (b < nJ) {
            const float bv = sm.Bf[b * 16 + col][kr];
#pragma unroll
            for (int e = 0; e < EW; ++e)
              acc[e][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                  xa[e], bv, acc[e][b], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // epilogue: the near and band tiers, scale, store both triangles.
  // FP32/BF16 16x16 MFMA result: D[i][j] at lane j + 16 (i / 4), reg i % 4.
  const double scale = 1.0 / (2.0 * S.a);
#pragma unroll
  for (int e = 0; e < EW; ++e) {
    const int el = wave * EW + e;
    const int eg = e0 + el;
    if (eg >= m) continue;
    const double Ee = E[eg];
    const int klo = sm.nlo[el], khi = sm.nhi[el];
    double *Re = Rbase + (int64_t)eg * estride;
#pragma unroll
    for (int b = 0; b < JMAX; ++b) {
      if (b >= nJ) continue;
      const int JB = JB0 + b;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = IB * 16 + 4 * kq + r;
        const int gj = JB * 16 + col;
        if (gi >= S.n || gj >= S.n) continue;
        if (JB == IB && gi > gj) continue;  // diagonal block: mirror the upper
        double v = (double)acc[e][b][r];
        for (int k = klo; k < khi; ++k) {
          const double diff = S.E_pole[k] - Ee;
          if (!(fabs(diff) < band)) continue;  // same test as the d_k staging
          const double wi = S.Wt[(int64_t)k * S.n_pad + gi];
          const double wj = S.Wt[(int64_t)k * S.n_pad + gj];
          if (fabs(diff) < delta)
            v += wi * wj / diff;
          else
            v += (double)(float)wi * (double)(float)wj * (double)(float)(1.0 / diff);
        }
        v *= scale;
        Re[(int64_t)gi * ld + gj] = v;
        Re[(int64_t)gj * ld + gi] = v;
      }
    }
  }
  __syncthreads();
}

template <bool BF16, int JMAX, int EW>
__global__ __launch_bounds__(256) void polesum_mixed_kernel(PsLaunch L) {
  __shared__ MxSmem<BF16, JMAX, EW> sm;
  __shared__ int s_item;
  const int tid = threadIdx.x;
  int it = -1;
  if (!L.counter) {
    const int chunk = (L.n_items + 7) / 8;
    it = (blockIdx.x % 8) * chunk + blockIdx.x / 8;
  }
  for (;;) {
    if (L.counter) {
      if (tid == 0) s_item = atomicAdd(L.counter, 1);
      __syncthreads();
      it = s_item;
      __syncthreads();
    }
    if (it >= L.n_items) break;
    const PsItem item = L.items[it];
    const SymDev &S = L.syms[item.sym];
    ps_mixed_item<BF16, JMAX, EW>(S, item.x, item.y, item.grp, L.E, L.m,
                                  L.delta, L.band,
                                  L.out.out + L.out.off[item.sym],
                                  L.out.estride, L.out.ld_mult * S.n, sm);
    if (!L.counter) break;
  }
}

template <bool BF16>
static hipError_t launch_mx(const PsLaunch &L, int variant, dim3 grid,
                            hipStream_t st) {
  switch (variant) {
    case PS_MX_J16_E8:
      hipLaunchKernelGGL((polesum_mixed_kernel<BF16, 16, 2>), grid, dim3(256),
                         0, st, L);
      break;
    case PS_MX_J8_E8:
      hipLaunchKernelGGL((polesum_mixed_kernel<BF16, 8, 2>), grid, dim3(256),
                         0, st, L);
      break;
    case PS_MX_J16_E4:
      hipLaunchKernelGGL((polesum_mixed_kernel<BF16, 16, 1>), grid, dim3(256),
                         0, st, L);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_polesum_mixed(const PsLaunch &L, int variant,
                                hipStream_t st) {
  unsigned grid;
  if (L.counter)
    grid = (unsigned)std::max(1, std::min(L.grid, L.n_items));
  else
    grid = (unsigned)(8 * ((L.n_items + 7) / 8));
  if (L.prec == RM_PREC_BF16X3) return launch_mx<true>(L, variant, dim3(grid), st);
  return launch_mx<false>(L, variant, dim3(grid), st);
}

}  // namespace rmx
