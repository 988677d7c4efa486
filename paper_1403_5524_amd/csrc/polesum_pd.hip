// Mixed-precision pole sum in pair-major form (paper Sec. 6, Eq. 1-2).
//
// For the upper-triangle channel pairs p = (i, j), i <= j, of one symmetry
//   R_p(E_e) = (1/2a) sum_k P_pk D_ke,   P_pk = w_ik w_jk,   D_ke = 1/(E_k - E_e)
// is one GEMM per symmetry, C[pairs x energies] = P[pairs x poles] D, with P
// formed once per symmetry (FP64 products, then rounded: FP32, or hi + lo
// BF16) and D generated inside the kernel from the pole and mesh energies
// (E_k - E_e from hi + lo FP32 splits of both energies, then one FP32
// reciprocal).  Poles with |E_k - E_e| < band get D = 0 here and are added
// in the epilogue: the near tier (< delta) from FP64 operands, the band tier
// from FP32-rounded w_ik, w_jk and D_ke with FP64 products and sum.
//
//   * FP32:       v_mfma_f32_16x16x4f32 on FP32 P and D;
//   * split BF16: P and D as hi + lo in BF16, Ph Dh + Ph Dl + Pl Dh with
//                 v_mfma_f32_16x16x32_bf16 (about 16 significant bits per
//                 product), FP32 accumulation.
//
// A workgroup computes a 256-pair x 128-energy tile (four wavefronts of
// 64 pairs x 128 energies); poles stream in chunks of 32 through
// double-buffered LDS: the next chunk's P rows are loaded into registers and
// its D block generated while the matrix cores work on the current one, with
// one barrier per chunk.  Work items (symmetry, pair block, energy block)
// are laid out pair-block-major and block b runs item (b mod 8) * ceil(N/8)
// + b / 8, so the energy blocks of one pair block run on one XCD and read
// its P rows through that XCD's L2.
#include <algorithm>

#include "rm_internal.h"

namespace rmx {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int PD_BM = 256;  // pairs per workgroup
constexpr int PD_BN = 128;  // energies per workgroup
constexpr int PD_KC = 32;   // poles per chunk

template <int PREC>
struct PdSmem;

template <>
struct PdSmem<RM_PREC_BF16X3> {
  // rows padded to 40 elements (80 B): 16-byte reads of 8 consecutive
  // lanes' rows fall on distinct banks
  __attribute__((aligned(16))) uint16_t Ah[2][PD_BM][PD_KC + 8];
  __attribute__((aligned(16))) uint16_t Al[2][PD_BM][PD_KC + 8];
  __attribute__((aligned(16))) uint16_t Bh[2][PD_BN][PD_KC + 8];
  __attribute__((aligned(16))) uint16_t Bl[2][PD_BN][PD_KC + 8];
  f2 Ep[3][PD_KC];  // pole energies (hi, lo) of three successive chunks
  f2 Ee2[PD_BN];    // the workgroup's energies (hi, lo)
  double Ee[PD_BN];
  int klo[PD_BN], khi[PD_BN];
};

template <>
struct PdSmem<RM_PREC_FP32> {
  // within a row, pole k = 4 s + q of the chunk sits at q * 8 + s, so a lane
  // reads its eight k-steps of one MFMA column as two 16-byte words
  __attribute__((aligned(16))) float A[2][PD_BM][PD_KC + 4];
  __attribute__((aligned(16))) float B[2][PD_BN][PD_KC + 4];
  f2 Ep[3][PD_KC];  // pole energies (hi, lo) of three successive chunks
  f2 Ee2[PD_BN];    // the workgroup's energies (hi, lo)
  double Ee[PD_BN];
  int klo[PD_BN], khi[PD_BN];
};

__device__ inline uint16_t bf16_bits(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ inline float bf16_value(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// x = hi + lo with hi, lo FP32 (lo carries the next 24 bits).
__device__ inline f2 pd_split(double x) {
  const float hi = (float)x;
  return f2{hi, (float)(x - (double)hi)};
}

// E_k - E_e from the (hi, lo) pairs in FP32: the hi difference is exact when
// the two are within a factor of two (otherwise the difference is large),
// so the result carries FP32 relative accuracy even for |E_k - E_e| ~ 1e-9 E.
__device__ inline float pd_diff(f2 ek, f2 ee) {
  return (ek.x - ee.x) + (ek.y - ee.y);
}

// The near-pole test; the D generation and the FP64 epilogue both use it, so
// every pole is summed exactly once.
__device__ inline bool pd_near(f2 ek, f2 ee, float delta) {
  return fabsf(pd_diff(ek, ee)) < delta;
}

__device__ inline int pd_lower_bound(const double *Ep, int nh, double x) {
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

// Staging registers of one P chunk: 16-byte words of the plane's own type.
template <int PREC>
struct PdReg {
  typedef u32x4 T;  // eight BF16
};
template <>
struct PdReg<RM_PREC_FP32> {
  typedef f4 T;
};

// P rows [row0, row0 + 256) x poles [k0, k0 + 32) into registers.
template <int PREC>
__device__ inline void pd_load_p(const SymDev &S, int row0, int k0,
                                 typename PdReg<PREC>::T (&r)[8]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int idx = tid + 256 * q;
    if constexpr (PREC == RM_PREC_BF16X3) {
      const int plane = idx >> 10, rem = idx & 1023;
      const int row = rem >> 2, piece = rem & 3;
      const uint16_t *src = plane ? S.Pl : S.Ph;
      r[q] = *(const u32x4 *)(src + (int64_t)(row0 + row) * S.nh_pad + k0 +
                              piece * 8);
    } else {
      const int row = idx >> 3, piece = idx & 7;
      r[q] = *(const f4 *)(S.P32 + (int64_t)(row0 + row) * S.nh_pad + k0 +
                           piece * 4);
    }
  }
}

template <int PREC>
__device__ inline void pd_store_p(PdSmem<PREC> &sm, int buf,
                                  const typename PdReg<PREC>::T (&r)[8]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int idx = tid + 256 * q;
    if constexpr (PREC == RM_PREC_BF16X3) {
      const int plane = idx >> 10, rem = idx & 1023;
      const int row = rem >> 2, piece = rem & 3;
      uint16_t *dst = plane ? &sm.Al[buf][row][piece * 8] : &sm.Ah[buf][row][piece * 8];
      *(u32x4 *)dst = r[q];
    } else {
      const int row = idx >> 3, piece = idx & 7;  // poles 4 piece .. +3
      float *dst = &sm.A[buf][row][0];
      const f4 v = r[q];
      dst[0 * 8 + piece] = v[0];
      dst[1 * 8 + piece] = v[1];
      dst[2 * 8 + piece] = v[2];
      dst[3 * 8 + piece] = v[3];
    }
  }
}

// D block of chunk c (pole energies in ring slot c % 3) for the workgroup's
// 128 energies: thread t forms energy t/2, poles 16 (t%2) .. +15.
template <int PREC>
__device__ inline void pd_gen_d(PdSmem<PREC> &sm, int buf, int c, int e0,
                                int m, float delta) {
  const int tid = threadIdx.x;
  const int el = tid >> 1, kh = (tid & 1) * 16;
  const bool ev = e0 + el < m;
  const f2 ee = sm.Ee2[el];
  const f2 *Ep = &sm.Ep[c % 3][kh];
  auto dval = [&](int u) -> float {
    const f2 ek = Ep[u];
    return (ev && !pd_near(ek, ee, delta))
               ? __builtin_amdgcn_rcpf(pd_diff(ek, ee))
               : 0.0f;
  };
  // scalar temporaries only (a private array here would be placed in LDS)
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const float v0 = dval(4 * g), v1 = dval(4 * g + 1);
    const float v2 = dval(4 * g + 2), v3 = dval(4 * g + 3);
    if constexpr (PREC == RM_PREC_BF16X3) {
      const uint16_t h0 = bf16_bits(v0), h1 = bf16_bits(v1);
      const uint16_t h2 = bf16_bits(v2), h3 = bf16_bits(v3);
      const uint16_t l0 = bf16_bits(v0 - bf16_value(h0));
      const uint16_t l1 = bf16_bits(v1 - bf16_value(h1));
      const uint16_t l2 = bf16_bits(v2 - bf16_value(h2));
      const uint16_t l3 = bf16_bits(v3 - bf16_value(h3));
      *(u32x2 *)&sm.Bh[buf][el][kh + 4 * g] =
          u32x2{(uint32_t)h0 | ((uint32_t)h1 << 16), (uint32_t)h2 | ((uint32_t)h3 << 16)};
      *(u32x2 *)&sm.Bl[buf][el][kh + 4 * g] =
          u32x2{(uint32_t)l0 | ((uint32_t)l1 << 16), (uint32_t)l2 | ((uint32_t)l3 << 16)};
    } else {
      // poles kh + 4g + c = 4 s + q: c is q, (kh / 4 + g) is s
      float *row = &sm.B[buf][el][0];
      const int s4 = (kh >> 2) + g;
      row[0 * 8 + s4] = v0;
      row[1 * 8 + s4] = v1;
      row[2 * 8 + s4] = v2;
      row[3 * 8 + s4] = v3;
    }
  }
}

// One chunk: issue chunk kc + 1's P rows into registers (the last chunk
// reloads itself, unused, so the loads stay unconditional), run chunk kc's
// MFMAs from LDS buffer kc % 2, then form chunk kc + 1's D block and store
// its P rows into the other buffer.
template <int PREC>
__device__ inline void pd_step(const SymDev &S, PdSmem<PREC> &sm,
                               f4 (&acc)[4][8], int kc, int nk, int row0,
                               int e0, int m, float delta32,
                               typename PdReg<PREC>::T (&pr)[8]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int cur = kc & 1, nxt = cur ^ 1;
  pd_load_p<PREC>(S, row0, min(kc + 1, nk - 1) * PD_KC, pr);
  // pole energies two chunks ahead, into the ring after the MFMAs
  double ep_next = 0.0;
  if (tid < PD_KC && kc + 2 < nk) ep_next = S.E_pole[(kc + 2) * PD_KC + tid];
    if constexpr (PREC == RM_PREC_BF16X3) {
      bf8 ah[4], al[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int r = wave * 64 + a * 16 + col;
        ah[a] = *(const bf8 *)&sm.Ah[cur][r][8 * kq];
        al[a] = *(const bf8 *)&sm.Al[cur][r][8 * kq];
      }
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int er = b * 16 + col;
        const bf8 bh = *(const bf8 *)&sm.Bh[cur][er][8 * kq];
        const bf8 bl = *(const bf8 *)&sm.Bl[cur][er][8 * kq];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh, acc[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < 4; ++a)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl, acc[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < 4; ++a)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh, acc[a][b], 0, 0, 0);
      }
    } else {
      f4 av[4][2];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int r = wave * 64 + a * 16 + col;
        av[a][0] = *(const f4 *)&sm.A[cur][r][kq * 8];
        av[a][1] = *(const f4 *)&sm.A[cur][r][kq * 8 + 4];
      }
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int er = b * 16 + col;
        const f4 b0 = *(const f4 *)&sm.B[cur][er][kq * 8];
        const f4 b1 = *(const f4 *)&sm.B[cur][er][kq * 8 + 4];
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
          for (int a = 0; a < 4; ++a)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                av[a][s >> 2][s & 3], s < 4 ? b0[s] : b1[s - 4], acc[a][b], 0,
                0, 0);
      }
    }
  if (kc + 1 < nk) {
    pd_gen_d<PREC>(sm, nxt, kc + 1, e0, m, delta32);
    pd_store_p<PREC>(sm, nxt, pr);
  }
  if (tid < PD_KC && kc + 2 < nk) sm.Ep[(kc + 2) % 3][tid] = pd_split(ep_next);
  __syncthreads();
}

template <int PREC>
__device__ void pd_item(const SymDev &S, int pb, int grp,
                        const double *__restrict__ E, int m, double delta,
                        double band, double *__restrict__ Rbase, int64_t estride, int ld,
                        PdSmem<PREC> &sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int row0 = pb * PD_BM;
  const int e0 = grp * PD_BN;
  const int nk = S.nh_pad / PD_KC;
  const float delta32 = (float)delta;
  const float band32 = (float)band;
  if (tid < PD_KC) {
    sm.Ep[0][tid] = pd_split(S.E_pole[tid]);
    if (nk > 1) sm.Ep[1][tid] = pd_split(S.E_pole[PD_KC + tid]);
  }
  if (tid < PD_BN) {
    const int e = e0 + tid;
    int lo = 0, hi = 0;
    double Ee = 0.0;
    if (e < m) {
      Ee = E[e];
      // superset of the near and band tiers; the epilogue applies the
      // exact tests
      lo = pd_lower_bound(S.E_pole, S.nh, Ee - 2.0 * band);
      hi = pd_lower_bound(S.E_pole, S.nh, Ee + 2.0 * band);
    }
    sm.Ee[tid] = Ee;
    sm.Ee2[tid] = pd_split(Ee);
    sm.klo[tid] = lo;
    sm.khi[tid] = hi;
  }
  __syncthreads();

  f4 acc[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};

  // chunk c sits in LDS buffer c % 2; chunk c + 1's P rows are in flight
  // in registers while chunk c's MFMAs run
  typename PdReg<PREC>::T pr[8];
  pd_load_p<PREC>(S, row0, 0, pr);
  pd_gen_d<PREC>(sm, 0, 0, e0, m, band32);
  pd_store_p<PREC>(sm, 0, pr);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) pd_step<PREC>(S, sm, acc, kc, nk, row0, e0, m, band32, pr);

  // epilogue: the near and band tiers, scale, store both triangles.
  // 16x16 FP32 MFMA result: D[i][j] at lane j + 16 (i / 4), register i % 4.
  const double scale = 1.0 / (2.0 * S.a);
  // this lane's 16 pairs (rows of its accumulators) and their channels
  int gij[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = row0 + wave * 64 + a * 16 + 4 * kq + r;
      gij[a][r] = p < S.np ? S.pair_ij[p] : -1;
    }
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const int el = b * 16 + col;
    const int e = e0 + el;
    if (e >= m) continue;
    const double Ee = sm.Ee[el];
    const f2 ee = sm.Ee2[el];
    const int klo = sm.klo[el], khi = sm.khi[el];
    double *Re = Rbase + (int64_t)e * estride;
    // the near and band tiers of this energy: one weight per pole, applied
    // to all 16 pairs
    double cor[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) cor[a][r] = 0.0;
    for (int k = klo; k < khi; ++k) {
      const double ek = S.E_pole[k];
      const float df = pd_diff(pd_split(ek), ee);
      if (!(fabsf(df) < band32)) continue;  // D's test: in the GEMM
      // near tier: FP64 operands; band tier: FP32-rounded operands
      const bool nr = fabsf(df) < delta32;
      const double t = nr ? 1.0 / (ek - Ee) : (double)__builtin_amdgcn_rcpf(df);
      const double *wk = S.Wt + (int64_t)k * S.n_pad;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ij = max(gij[a][r], 0);
          const double wi = wk[ij >> 16], wj = wk[ij & 0xffff];
          const double x = nr ? wi : (double)(float)wi;
          const double y = nr ? wj : (double)(float)wj;
          cor[a][r] = fma(x * y, t, cor[a][r]);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ij = gij[a][r];
        if (ij < 0) continue;
        const int gi = ij >> 16, gj = ij & 0xffff;
        const double v = ((double)acc[a][b][r] + cor[a][r]) * scale;
        Re[(int64_t)gi * ld + gj] = v;
        if (gi != gj) Re[(int64_t)gj * ld + gi] = v;
      }
  }
  __syncthreads();
}

template <int PREC>
__global__ __launch_bounds__(256) void polesum_pd_kernel(PsLaunch L) {
  __shared__ PdSmem<PREC> sm;
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
    pd_item<PREC>(S, item.x, item.grp, L.E, L.m, L.delta, L.band,
                  L.out.out + L.out.off[item.sym], L.out.estride,
                  L.out.ld_mult * S.n, sm);
    if (!L.counter) break;
  }
}

hipError_t launch_polesum_pd(const PsLaunch &L, hipStream_t st) {
  unsigned grid;
  if (L.counter)
    grid = (unsigned)std::max(1, std::min(L.grid, L.n_items));
  else
    grid = (unsigned)(8 * ((L.n_items + 7) / 8));
  if (L.prec == RM_PREC_BF16X3)
    hipLaunchKernelGGL(polesum_pd_kernel<RM_PREC_BF16X3>, dim3(grid), dim3(256),
                       0, st, L);
  else if (L.prec == RM_PREC_FP32)
    hipLaunchKernelGGL(polesum_pd_kernel<RM_PREC_FP32>, dim3(grid), dim3(256),
                       0, st, L);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---- pair products P_pk = w_ik w_jk, formed once per symmetry ----

template <int PREC>
__global__ void pd_build_kernel(const double *__restrict__ Wt, int n_pad,
                                const int32_t *__restrict__ pair_ij, int np,
                                int np_pad, int nh_pad, uint16_t *Ph,
                                uint16_t *Pl, float *P32) {
  const int64_t total = (int64_t)np_pad * nh_pad;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(q / nh_pad), k = (int)(q % nh_pad);
    double v = 0.0;
    if (p < np) {
      const int ij = pair_ij[p];
      v = Wt[(int64_t)k * n_pad + (ij >> 16)] * Wt[(int64_t)k * n_pad + (ij & 0xffff)];
    }
    if (PREC == RM_PREC_BF16X3) {
      const uint16_t h = bf16_bits((float)v);
      Ph[q] = h;
      Pl[q] = bf16_bits((float)(v - (double)bf16_value(h)));
    } else {
      P32[q] = (float)v;
    }
  }
}

hipError_t launch_pd_build(const Sym &s, int prec, hipStream_t st) {
  const int64_t total = (int64_t)s.np_pad * s.nh_pad;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  if (prec == RM_PREC_BF16X3)
    hipLaunchKernelGGL(pd_build_kernel<RM_PREC_BF16X3>, dim3(grid), dim3(256), 0,
                       st, s.Wt, s.n_pad, s.pair_ij, s.np, s.np_pad, s.nh_pad,
                       s.Ph, s.Pl, (float *)nullptr);
  else
    hipLaunchKernelGGL(pd_build_kernel<RM_PREC_FP32>, dim3(grid), dim3(256), 0,
                       st, s.Wt, s.n_pad, s.pair_ij, s.np, s.np_pad, s.nh_pad,
                       (uint16_t *)nullptr, (uint16_t *)nullptr, s.P32);
  return hipGetLastError();
}

}  // namespace rmx

// ---------------------------------------------------------------------------
// FP64 pair-major pole sum: the same GEMM with P and D in FP64
// (v_mfma_f64_16x16x4f64), every pole in the product (no near split).  A
// workgroup computes 256 pairs x 64 energies (four wavefronts of 64 x 64)
// over chunks of 16 poles; within a row, pole k = 4 s + q of a chunk sits at
// q * 4 + s so a lane reads its four k-steps as two 16-byte words.

namespace rmx {

constexpr int PD64_BN = 64;  // energies per workgroup
constexpr int PD64_KC = 16;  // poles per chunk

struct Pd64Smem {
  __attribute__((aligned(16))) double A[2][PD_BM][PD64_KC + 2];
  __attribute__((aligned(16))) double B[2][PD64_BN][PD64_KC + 2];
  double Ep[3][PD64_KC];
  double Ee[PD64_BN];
};

typedef double d4x __attribute__((ext_vector_type(4)));
typedef double d2x __attribute__((ext_vector_type(2)));

__device__ inline void pd64_load_p(const SymDev &S, int row0, int k0,
                                   d2x (&r)[8]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int idx = tid + 256 * q;
    const int row = idx >> 3, piece = idx & 7;  // poles 2 piece, 2 piece + 1
    r[q] = *(const d2x *)(S.P64 + (int64_t)(row0 + row) * S.nh_pad + k0 +
                          piece * 2);
  }
}

__device__ inline void pd64_store_p(Pd64Smem &sm, int buf, const d2x (&r)[8]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int idx = tid + 256 * q;
    const int row = idx >> 3, piece = idx & 7;
    const int k0 = 2 * piece, k1 = k0 + 1;
    const d2x v = r[q];
    sm.A[buf][row][(k0 & 3) * 4 + (k0 >> 2)] = v[0];
    sm.A[buf][row][(k1 & 3) * 4 + (k1 >> 2)] = v[1];
  }
}

// D of chunk c for the workgroup's 64 energies: thread t forms energy t/4,
// poles 4 (t%4) .. +3, in FP64.
__device__ inline void pd64_gen_d(Pd64Smem &sm, int buf, int c, int e0, int m) {
  const int tid = threadIdx.x;
  const int el = tid >> 2, k4 = (tid & 3) * 4;
  const bool ev = e0 + el < m;
  const double Ee = sm.Ee[el];
  double *row = &sm.B[buf][el][0];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = k4 + u;
    row[(k & 3) * 4 + (k >> 2)] = ev ? 1.0 / (sm.Ep[c % 3][k] - Ee) : 0.0;
  }
}

__device__ inline void pd64_step(const SymDev &S, Pd64Smem &sm,
                                 d4x (&acc)[4][4], int kc, int nk, int row0,
                                 int e0, int m, d2x (&pr)[8]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int cur = kc & 1, nxt = cur ^ 1;
  pd64_load_p(S, row0, min(kc + 1, nk - 1) * PD64_KC, pr);
  double ep_next = 0.0;
  if (tid < PD64_KC && kc + 2 < nk) ep_next = S.E_pole[(kc + 2) * PD64_KC + tid];
  d4x av[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = wave * 64 + a * 16 + col;
    const d2x lo = *(const d2x *)&sm.A[cur][r][kq * 4];
    const d2x hi = *(const d2x *)&sm.A[cur][r][kq * 4 + 2];
    av[a] = d4x{lo[0], lo[1], hi[0], hi[1]};
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int er = b * 16 + col;
    const d2x lo = *(const d2x *)&sm.B[cur][er][kq * 4];
    const d2x hi = *(const d2x *)&sm.B[cur][er][kq * 4 + 2];
    const d4x bv = d4x{lo[0], lo[1], hi[0], hi[1]};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int a = 0; a < 4; ++a)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][s], bv[s],
                                                          acc[a][b], 0, 0, 0);
  }
  if (kc + 1 < nk) {
    pd64_gen_d(sm, nxt, kc + 1, e0, m);
    pd64_store_p(sm, nxt, pr);
  }
  if (tid < PD64_KC && kc + 2 < nk) sm.Ep[(kc + 2) % 3][tid] = ep_next;
  __syncthreads();
}

__device__ void pd64_item(const SymDev &S, int pb, int grp,
                          const double *__restrict__ E, int m,
                          double *__restrict__ Rbase, int64_t estride, int ld,
                          Pd64Smem &sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int row0 = pb * PD_BM;
  const int e0 = grp * PD64_BN;
  const int nk = S.nh_pad / PD64_KC;
  if (tid < PD64_KC) {
    sm.Ep[0][tid] = S.E_pole[tid];
    if (nk > 1) sm.Ep[1][tid] = S.E_pole[PD64_KC + tid];
  }
  if (tid < PD64_BN) sm.Ee[tid] = e0 + tid < m ? E[e0 + tid] : 0.0;
  __syncthreads();
  d4x acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4x{0.0, 0.0, 0.0, 0.0};
  d2x pr[8];
  pd64_load_p(S, row0, 0, pr);
  pd64_gen_d(sm, 0, 0, e0, m);
  pd64_store_p(sm, 0, pr);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) pd64_step(S, sm, acc, kc, nk, row0, e0, m, pr);

  // FP64 16x16x4 result: D[i][j] at j = lane % 16, i = lane / 16 + 4 r
  const double scale = 1.0 / (2.0 * S.a);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int e = e0 + b * 16 + col;
    if (e >= m) continue;
    double *Re = Rbase + (int64_t)e * estride;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = row0 + wave * 64 + a * 16 + kq + 4 * r;
        if (p >= S.np) continue;
        const int ij = S.pair_ij[p];
        const int gi = ij >> 16, gj = ij & 0xffff;
        const double v = acc[a][b][r] * scale;
        Re[(int64_t)gi * ld + gj] = v;
        if (gi != gj) Re[(int64_t)gj * ld + gi] = v;
      }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void polesum_pd64_kernel(PsLaunch L) {
  __shared__ Pd64Smem sm;
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
    pd64_item(S, item.x, item.grp, L.E, L.m, L.out.out + L.out.off[item.sym],
              L.out.estride, L.out.ld_mult * S.n, sm);
    if (!L.counter) break;
  }
}

hipError_t launch_polesum_pd64(const PsLaunch &L, hipStream_t st) {
  unsigned grid;
  if (L.counter)
    grid = (unsigned)std::max(1, std::min(L.grid, L.n_items));
  else
    grid = (unsigned)(8 * ((L.n_items + 7) / 8));
  hipLaunchKernelGGL(polesum_pd64_kernel, dim3(grid), dim3(256), 0, st, L);
  return hipGetLastError();
}

__global__ void pd64_build_kernel(const double *__restrict__ Wt, int n_pad,
                                  const int32_t *__restrict__ pair_ij, int np,
                                  int np_pad, int nh_pad, double *P64) {
  const int64_t total = (int64_t)np_pad * nh_pad;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(q / nh_pad), k = (int)(q % nh_pad);
    double v = 0.0;
    if (p < np) {
      const int ij = pair_ij[p];
      v = Wt[(int64_t)k * n_pad + (ij >> 16)] * Wt[(int64_t)k * n_pad + (ij & 0xffff)];
    }
    P64[q] = v;
  }
}

hipError_t launch_pd64_build(const Sym &s, hipStream_t st) {
  const int64_t total = (int64_t)s.np_pad * s.nh_pad;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(pd64_build_kernel, dim3(grid), dim3(256), 0, st, s.Wt,
                     s.n_pad, s.pair_ij, s.np, s.np_pad, s.nh_pad, s.P64);
  return hipGetLastError();
}

}  // namespace rmx
