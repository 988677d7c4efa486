// Dipole pole sum of the photoionization path: at every energy of a chunk
//     g_i(E) = (1/sqrt2) sum_k w_ik d_k / (E_k - E),
// the vector that turns the matching solution into bound-free dipole
// amplitudes (the inner-region expansion of the continuum, Bloch b = 0, in
// the convention R_ij = (1/2a) sum_k w_ik w_jk / (E_k - E)).  It is the
// pole sum of Sec. 6, Eq. 1-2, with the second factor W replaced by one
// dipole vector: an (n x N_H) by (N_H x m) product on the FP64 matrix cores
// whose right operand d_k / (E_k - E) is formed in LDS, one stage of 16
// poles at a time, and shared by the four waves (16 channels each) of a
// workgroup of 64 channels x 64 energies.
#include "rm_internal.h"

namespace rmx {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int DP_BE = 64;  // energies per workgroup
constexpr int DP_KC = 16;  // poles per stage

__global__ __launch_bounds__(256) void dip_polesum_kernel(
    SymDev S, const double *__restrict__ E, int m, double *__restrict__ out,
    int64_t estride, int64_t off, int part) {
  __shared__ double D[DP_KC][DP_BE];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i0 = blockIdx.x * 64 + 16 * wave;
  const int e0 = blockIdx.y * DP_BE;
  const int col = lane & 15, kq = lane >> 4;
  // D staging: energy e0 + (tid % 64), poles (tid / 64) + 4 u of a stage
  const int se = e0 + (tid & 63);
  const bool ev = se < m;
  const double Ee = ev ? E[se] : 0.0;
  const int sk = tid >> 6;
  const bool iv = i0 + col < S.n_pad;
  const double *wrow = S.Wt + (iv ? i0 + col : 0);

  d4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < S.nh_pad; k0 += DP_KC) {
    double dv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + sk + 4 * u;
      // part 0: d_k / (E_k - E); 1, 2: real and imaginary part of
      // d_k / (E_k - i Gamma_k/2 - E)
      const double x = S.E_pole[k] - Ee;
      double v;
      if (part == 0) {
        v = S.dip[k] / x;
      } else {
        const double h = 0.5 * S.gam[k];
        v = S.dip[k] * (part == 1 ? x : h) / fma(x, x, h * h);
      }
      dv[u] = ev ? v : 0.0;
    }
    // A[i][k] = w_ik for i = i0 + col, k = k0 + 4 s + kq
    double a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double w = wrow[(int64_t)(k0 + 4 * s + kq) * S.n_pad];
      a[s] = iv ? w : 0.0;
    }
    __syncthreads();  // the previous stage has been read
#pragma unroll
    for (int u = 0; u < 4; ++u) D[sk + 4 * u][tid & 63] = dv[u];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(
            a[s], D[4 * s + kq][16 * b + col], acc[b], 0, 0, 0);
  }
  // FP64 16x16x4 result: lane holds row kq + 4 r (channel), column col
  // (energy) of block b
  const double rs2 = 0.70710678118654752440;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + kq + 4 * r, e = e0 + 16 * b + col;
      if (i < S.n && e < m) out[(int64_t)e * estride + off + i] = acc[b][r] * rs2;
    }
}

hipError_t launch_dip_polesum(const SymDev &S, const double *E, int m,
                              double *out, int64_t estride, int64_t off,
                              hipStream_t st, int part) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((S.n + 63) / 64), (unsigned)((m + DP_BE - 1) / DP_BE));
  hipLaunchKernelGGL(dip_polesum_kernel, grid, dim3(256), 0, st, S, E, m, out,
                     estride, off, part);
  return hipGetLastError();
}

}  // namespace rmx
