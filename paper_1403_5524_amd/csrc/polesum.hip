// Pole-sum contraction (paper Sec. 6, Eq. 1-2), FP64, on gfx950 matrix
// cores, grouped over every symmetry of a chunk.
//
// R(E) = (1/2a) W diag(d(E)) W^T with d_k(E) = 1/(E_k - E): per energy a
// symmetric n x n product whose operand W (n x N_H) is shared by every
// energy.  A work item is one upper-triangle tile pair (I, J) of 32 x 32
// outputs of one symmetry and a group of 16 energies; W tiles of 32 poles
// are staged in LDS once and reused by all 16 energies, each wave scaling
// the A fragment by its own d_k(E) before the MFMA.  The mirror block is
// written from the same accumulators.
//
// Items come from a table built on the host (largest symmetries first).
// Without a counter, block b runs item (b mod 8) * ceil(N/8) + b / 8, so
// consecutive items -- the same W tiles for successive energy groups -- land
// on the same XCD (blocks are dispatched round-robin over the 8 XCDs) and
// share its L2.  With a counter the grid is persistent and pulls items.
#include <algorithm>

#include "rm_internal.h"

namespace rmx {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int PS_T = 32;    // output tile edge
constexpr int PS_KC = 32;   // poles per LDS stage
constexpr int PS_EW = 4;    // energies per wave
constexpr int PS_EG = 16;   // energies per workgroup (4 waves)

struct F64Smem {  // two stages: one feeds the MFMAs while the next fills
  double As[2][PS_KC][PS_T];
  double Bs[2][PS_KC][PS_T];
  double Ds[2][PS_EG][PS_KC];
};

// One work item: tile pair (I, J), J >= I, for PS_EG energies.  MASK bit
// 2 a + b says whether the 16 x 16 output block (a, b) of the 32 x 32 tile
// holds any element that is kept (row and column below n, row <= column on
// a diagonal tile); the others are never formed.  Diagonal tiles are
// exactly the masks without block (1, 0).
// Pole weight of part PART (see PsLaunch::part) for pole energy ep, width
// gm and energy e: 1/(ep - e), or the real / imaginary part of
// 1/(ep - i gm/2 - e) = (x + i h)/(x^2 + h^2), x = ep - e, h = gm/2.
template <int PART>
__device__ inline double ps_weight(double ep, double gm, double e) {
  const double x = ep - e;
  if constexpr (PART == 0) {
    return 1.0 / x;
  } else {
    const double h = 0.5 * gm;
    return (PART == 1 ? x : h) / fma(x, x, h * h);
  }
}

template <int MASK, int PART>
__device__ void ps_f64_item_m(const SymDev &S, int I, int J, int grp,
                              const double *__restrict__ E, int m,
                              double *__restrict__ Rbase, int64_t estride,
                              int ld, F64Smem &sm) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int e0 = grp * PS_EG;
  constexpr bool diag = !(MASK & 4);
  const int n_pad = S.n_pad;

  const int ld_k = tid >> 3;       // staging: 8 threads per pole row
  const int ld_c = (tid & 7) * 4;  // 4 doubles each
  const double *wa = S.Wt + (int64_t)ld_k * n_pad + I * PS_T + ld_c;
  const double *wb = S.Wt + (int64_t)ld_k * n_pad + J * PS_T + ld_c;
  double Eloc[2];
  int dk[2], de[2];
  bool ev[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int idx = tid + 256 * u;
    de[u] = idx / PS_KC;
    dk[u] = idx % PS_KC;
    const int e = e0 + de[u];
    ev[u] = e < m;
    Eloc[u] = ev[u] ? E[e] : 0.0;
  }

  d4 acc[PS_EW][2][2];
#pragma unroll
  for (int e = 0; e < PS_EW; ++e)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[e][a][b] = d4{0.0, 0.0, 0.0, 0.0};

  const int col = lane & 15;
  const int kq = lane >> 4;

  double2 ra0 = *(const double2 *)(wa);
  double2 ra1 = *(const double2 *)(wa + 2);
  double2 rb0 = ra0, rb1 = ra1;
  if (!diag) {
    rb0 = *(const double2 *)(wb);
    rb1 = *(const double2 *)(wb + 2);
  }
  double ep0 = S.E_pole[dk[0]], ep1 = S.E_pole[dk[1]];
  double gm0 = 0.0, gm1 = 0.0;
  if constexpr (PART != 0) {
    gm0 = S.gam[dk[0]];
    gm1 = S.gam[dk[1]];
  }
  // stage chunk c (held in registers) into LDS buffer c % 2
  auto stage = [&](int buf) {
    *(double2 *)&sm.As[buf][ld_k][ld_c] = ra0;
    *(double2 *)&sm.As[buf][ld_k][ld_c + 2] = ra1;
    if (!diag) {
      *(double2 *)&sm.Bs[buf][ld_k][ld_c] = rb0;
      *(double2 *)&sm.Bs[buf][ld_k][ld_c + 2] = rb1;
    }
    sm.Ds[buf][de[0]][dk[0]] = ev[0] ? ps_weight<PART>(ep0, gm0, Eloc[0]) : 0.0;
    sm.Ds[buf][de[1]][dk[1]] = ev[1] ? ps_weight<PART>(ep1, gm1, Eloc[1]) : 0.0;
  };
  // load chunk starting at pole kn into registers
  auto fetch = [&](int kn) {
    const int64_t off = (int64_t)kn * n_pad;
    ra0 = *(const double2 *)(wa + off);
    ra1 = *(const double2 *)(wa + off + 2);
    if (!diag) {
      rb0 = *(const double2 *)(wb + off);
      rb1 = *(const double2 *)(wb + off + 2);
    }
    ep0 = S.E_pole[kn + dk[0]];
    ep1 = S.E_pole[kn + dk[1]];
    if constexpr (PART != 0) {
      gm0 = S.gam[kn + dk[0]];
      gm1 = S.gam[kn + dk[1]];
    }
  };
  stage(0);
  if (PS_KC < S.nh_pad) fetch(PS_KC);
  __syncthreads();

  int buf = 0;
  for (int k0 = 0; k0 < S.nh_pad; k0 += PS_KC, buf ^= 1) {
    const double(*As)[PS_T] = sm.As[buf];
    const double(*Bsel)[PS_T] = diag ? sm.As[buf] : sm.Bs[buf];
    const double(*Ds)[PS_KC] = sm.Ds[buf];
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
        if constexpr (MASK & 1)
          acc[e][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa0, b0, acc[e][0][0], 0, 0, 0);
        if constexpr (MASK & 2)
          acc[e][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa0, b1, acc[e][0][1], 0, 0, 0);
        if constexpr (MASK & 4)
          acc[e][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa1, b0, acc[e][1][0], 0, 0, 0);
        if constexpr (MASK & 8)
          acc[e][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa1, b1, acc[e][1][1], 0, 0, 0);
      }
    }
    // the next chunk (already in registers) into the other buffer, then
    // start loading the one after it; one barrier per chunk
    if (k0 + PS_KC < S.nh_pad) {
      stage(buf ^ 1);
      if (k0 + 2 * PS_KC < S.nh_pad) fetch(k0 + 2 * PS_KC);
    }
    __syncthreads();
  }

  // FP64 16x16x4 MFMA result: lane holds D[i][j] with j = lane % 16 and
  // i = lane / 16 + 4 r (rows interleaved across the four result registers;
  // the FP32/BF16 forms use i = 4 (lane / 16) + r).
  const double scale = 1.0 / (2.0 * S.a);
#pragma unroll
  for (int e = 0; e < PS_EW; ++e) {
    const int eg = e0 + wave * PS_EW + e;
    if (eg >= m) continue;
    double *Re = Rbase + (int64_t)eg * estride;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (!(MASK & (1 << (2 * a + b)))) continue;  // compile-time
          const int gi = I * PS_T + a * 16 + kq + 4 * r;
          const int gj = J * PS_T + b * 16 + col;
          // diagonal tiles: the upper triangle is mirrored so R is exactly
          // symmetric
          if (gi < S.n && gj < S.n && (!diag || gi <= gj)) {
            const double v = acc[e][a][b][r] * scale;
            Re[(int64_t)gi * ld + gj] = v;
            Re[(int64_t)gj * ld + gi] = v;
          }
        }
  }
}

template <int PART>
__device__ void ps_f64_item(const SymDev &S, int I, int J, int grp,
                            const double *__restrict__ E, int m,
                            double *__restrict__ Rbase, int64_t estride,
                            int ld, F64Smem &sm) {
  // the last tile may reach at most 16 rows past n (n_pad = 32 ceil(n/32))
  if (I == J) {
    if (S.n - I * PS_T <= 16)
      ps_f64_item_m<1, PART>(S, I, J, grp, E, m, Rbase, estride, ld, sm);
    else
      ps_f64_item_m<1 | 2 | 8, PART>(S, I, J, grp, E, m, Rbase, estride, ld, sm);
  } else {
    if (S.n - J * PS_T <= 16)
      ps_f64_item_m<1 | 4, PART>(S, I, J, grp, E, m, Rbase, estride, ld, sm);
    else
      ps_f64_item_m<15, PART>(S, I, J, grp, E, m, Rbase, estride, ld, sm);
  }
}

// two workgroups per CU (41 KB of LDS and at most 256 registers per lane
// each), so one's barrier and staging overlap the other's MFMAs
template <int PART>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void polesum_f64_kernel(PsLaunch L) {
  __shared__ F64Smem sm;
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
    ps_f64_item<PART>(S, item.x, item.y, item.grp, L.E, L.m,
                L.out.out + L.out.off[item.sym], L.out.estride,
                L.out.ld_mult * S.n, sm);
    if (!L.counter) break;
  }
}

hipError_t launch_polesum_mixed(const PsLaunch &L, int variant, hipStream_t st);

int ps_energy_group(int variant) {
  switch (variant) {
    case PS_F64_T32_E16: return PS_EG;
    case PS_MX_J16_E8: return 8;
    case PS_MX_J8_E8: return 8;
    case PS_MX_J16_E4: return 4;
    case PS_PD: return 128;
    case PS_PD64: return 64;
  }
  return 1;
}

void ps_tiles(const Sym &s, int variant, std::vector<std::pair<int, int>> &out) {
  out.clear();
  if (variant == PS_F64_T32_E16) {
    const int nt = s.n_pad / PS_T;
    for (int I = 0; I < nt; ++I)
      for (int J = I; J < nt; ++J) out.push_back({I, J});
    return;
  }
  if (variant == PS_PD || variant == PS_PD64) {
    for (int pb = 0; pb < s.np_pad / kPairBlock; ++pb) out.push_back({pb, 0});
    return;
  }
  const int jmax = (variant == PS_MX_J8_E8) ? 8 : 16;
  const int nblk = s.n_pad / 16;
  for (int IB = 0; IB < nblk; ++IB)
    for (int JB0 = IB; JB0 < nblk; JB0 += jmax) out.push_back({IB, JB0});
}

hipError_t launch_polesum(const PsLaunch &L, int variant, hipStream_t st) {
  if (L.n_items <= 0 || L.m <= 0) return hipSuccess;
  if (variant == PS_PD) return launch_polesum_pd(L, st);
  if (variant == PS_PD64) return launch_polesum_pd64(L, st);
  if (variant != PS_F64_T32_E16) return launch_polesum_mixed(L, variant, st);
  unsigned grid;
  if (L.counter)
    grid = (unsigned)std::max(1, std::min(L.grid, L.n_items));
  else
    grid = (unsigned)(8 * ((L.n_items + 7) / 8));
  if (L.part == 1)
    hipLaunchKernelGGL(polesum_f64_kernel<1>, dim3(grid), dim3(256), 0, st, L);
  else if (L.part == 2)
    hipLaunchKernelGGL(polesum_f64_kernel<2>, dim3(grid), dim3(256), 0, st, L);
  else
    hipLaunchKernelGGL(polesum_f64_kernel<0>, dim3(grid), dim3(256), 0, st, L);
  return hipGetLastError();
}

}  // namespace rmx
