// Inner-region step: the poles E_k and surface amplitudes w_ik the sweep
// consumes, from the full eigen-solve of an inner-region Hamiltonian (the
// paper diagonalises each symmetry's Hamiltonian completely, Sec. 2-3).  A
// multichannel model stands in for the unpublished atomic Hamiltonians: on
// [0, a] the channel functions obey
//     u_i'' = sum_j [(l_i (l_i + 1)/r^2 - 2z/r + e_i - E) delta_ij + U_ij] u_j,
//     U_ij(r) = -depth_ij exp(-(r / range_ij)^2),
// expanded per channel in phi_m(r) = sqrt(2/a) sin(kappa_m r), kappa_m a =
// (m + 1/2) pi (u(0) = 0, u'(a) = 0: the Bloch term with b = 0 vanishes and
// the kinetic part is diag(kappa_m^2)).  Matrix elements of the potential by
// Gauss-Legendre quadrature; the symmetric eigenproblem by one-sided
// (Hestenes) Jacobi on H + sigma I (sigma from Gershgorin, so the matrix is
// positive definite): rotations V make its columns mutually orthogonal, and
// then column k is (H + sigma I) v_k with v_k an eigenvector.  The rotations
// act on pairs of 16-column blocks (Gram matrix by FP64 MFMA, its 32 x 32
// eigenproblem in LDS, the block rotation applied by FP64 MFMA), so a sweep
// reads the matrix nb - 1 times for nb = D / 16 blocks rather than D - 1.
// w_ik = sqrt2 sum_m V_(i,m),k phi_m(a) with phi_m(a) = sqrt(2/a) (-1)^m,
// the convention of R = (1/2a) sum_k w_ik w_jk / (E_k - E).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "rm_internal.h"

namespace rmx {

const char *set_error(int code, const char *msg);  // defined in rm_api.hip

static int in_fail(int code, const std::string &msg) {
  set_error(code, msg.c_str());
  return code;
}

typedef double d4 __attribute__((ext_vector_type(4)));

// Tables of the quadrature, Qp = Q rounded up to a multiple of 4 with zero
// entries beyond Q: phi[m][q] = sqrt(2/a) sin(kappa_m r_q) and
// wv[i][j][q] = w_q W_ij(r_q) (W without E).
__global__ void inner_tables_kernel(int n, int N, int Q, int Qp, double a, double z,
                                    const double *__restrict__ rq,
                                    const double *__restrict__ wq,
                                    const double *__restrict__ e_thr,
                                    const int32_t *__restrict__ l,
                                    const double *__restrict__ depth,
                                    const double *__restrict__ range,
                                    double *__restrict__ phi,
                                    double *__restrict__ wv) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nphi = (int64_t)N * Qp, nw = (int64_t)n * n * Qp;
  if (idx < nphi) {
    const int m = (int)(idx / Qp), q = (int)(idx % Qp);
    phi[idx] = q < Q ? sqrt(2.0 / a) * sin((m + 0.5) * M_PI / a * rq[q]) : 0.0;
  } else if (idx < nphi + nw) {
    const int64_t t = idx - nphi;
    const int ij = (int)(t / Qp), q = (int)(t % Qp);
    if (q >= Q) {
      wv[t] = 0.0;
      return;
    }
    const int i = ij / n, j = ij % n;
    const double r = rq[q], x = r / range[ij];
    double v = -depth[ij] * exp(-x * x);
    if (i == j) v += l[i] * (l[i] + 1.0) / (r * r) - 2.0 * z / r + e_thr[i];
    wv[t] = wq[q] * v;
  }
}

// H[p][p'] (column-major, leading dimension ld) for p = i N + m:
// kappa_m^2 delta + sum_q phi_m(r_q) w_q W_ij(r_q) phi_m'(r_q), i.e. the
// block (i, j) is Phi diag(wv_ij) Phi^T, a product on the FP64 matrix cores.
// One wavefront per 32 x 32 tile (block pair (i, j) = (blockIdx.x / n,
// blockIdx.x % n), tile row blockIdx.y, tile column blockIdx.z); only the
// lower triangle of H is computed (blocks i > j whole, the diagonal blocks'
// tiles tr >= tc, and in those only row >= column), each value written to
// both halves so that H is exactly symmetric.  MFMA 16x16x4: lane (col, kq) holds phi[m0 + col]
// [q0 + kq] (times wv for the A operand), k = the quadrature node.
__global__ __launch_bounds__(64) void inner_assemble_kernel(
    int n, int N, int Qp, double a, const double *__restrict__ phi,
    const double *__restrict__ wv, double *__restrict__ H, int ld) {
  const int tr = blockIdx.y, tc = blockIdx.z;
  const int i = blockIdx.x / n, j = blockIdx.x % n;
  if (j > i || (i == j && tc > tr)) return;
  const int lane = threadIdx.x, col = lane & 15, kq = lane >> 4;
  const int m0 = tr * 32, c0 = tc * 32;
  // rows beyond N read row N - 1 and are masked out
  const int ra0 = min(m0 + col, N - 1), ra1 = min(m0 + 16 + col, N - 1);
  const int rb0 = min(c0 + col, N - 1), rb1 = min(c0 + 16 + col, N - 1);
  const double *pa0 = phi + (int64_t)ra0 * Qp + kq, *pa1 = phi + (int64_t)ra1 * Qp + kq;
  const double *pb0 = phi + (int64_t)rb0 * Qp + kq, *pb1 = phi + (int64_t)rb1 * Qp + kq;
  const double *pw = wv + (int64_t)(i * n + j) * Qp + kq;
  d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  for (int q0 = 0; q0 < Qp; q0 += 4) {
    const double wq = pw[q0];
    const double a0 = pa0[q0] * wq, a1 = pa1[q0] * wq;
    const double b0 = pb0[q0], b1 = pb1[q0];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  // output lane r: row m0 + 16 x + kq + 4 r, column c0 + 16 y + col
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + 16 * x + kq + 4 * r, mp = c0 + 16 * y + col;
        if (m >= N || mp >= N) continue;
        const int64_t row = (int64_t)i * N + m, cl = (int64_t)j * N + mp;
        if (row < cl) continue;
        double v = acc[x][y][r];
        if (row == cl) {
          const double km = (m + 0.5) * M_PI / a;
          v += km * km;
        }
        H[cl * ld + row] = v;
        H[row * ld + cl] = v;
      }
}

// Row-wise Gershgorin lower bounds H_rr - sum_{c != r} |H_rc|.
__global__ void inner_gershgorin_kernel(const double *__restrict__ H, int D,
                                        int ld, double *lb) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D) return;
  double s = 0.0;
  for (int c = 0; c < D; ++c)
    if (c != r) s += fabs(H[(int64_t)c * ld + r]);
  lb[r] = H[(int64_t)r * ld + r] - s;
}

// A = H + sigma I in its leading D x D block, the padding rows and columns
// (up to Dp) zero; V = I.
__global__ void inner_init_kernel(double *A, double *V, int D, int Dp,
                                  double sigma) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)Dp * Dp) return;
  const int64_t c = idx / Dp, r = idx % Dp;
  if (c >= D || r >= D) A[idx] = 0.0;
  else if (r == c) A[idx] += sigma;
  V[idx] = (r == c) ? 1.0 : 0.0;
}

// Blocked one-sided Jacobi.  The Dp columns (Dp a multiple of 32) form
// nb = Dp / 16 blocks; in round-robin step t every block pair (P, Q) of the
// circle method ((t, nb - 1) for k = 0, else (t + k, t - k) mod (nb - 1))
// is handled at once: its 32 columns X give the Gram matrix G = X^T X, the
// eigenvectors U of G (two-sided Jacobi in LDS) make X U mutually
// orthogonal, and X <- X U, V <- V U.  Every column pair meets in some block
// pair each sweep, so a sweep in which no Gram fails the test
// |G_pq| <= tol sqrt(G_pp G_qq) leaves all columns mutually orthogonal.
constexpr int BJ_B = 16;        // columns per block
constexpr int BJ_W = 2 * BJ_B;  // columns per block pair
constexpr int BJ_CH = 256;      // rows per rotation workgroup (4 waves x 64)
constexpr int BJ_MAXCH = 16;    // row chunks of the Gram kernel, at most
constexpr int BJ_DMAX = 16384;  // largest dimension

__device__ inline void bj_pair(int nb, int t, int k, int &P, int &Qb) {
  const int L = nb - 1;
  if (k == 0) {
    P = t % L;
    Qb = L;
  } else {
    P = (t + k) % L;
    Qb = (t - k + L) % L;
  }
}

// column of A (or V) at position c in [0, 32) of block pair (P, Qb)
__device__ inline int bj_col(int P, int Qb, int c) {
  return c < BJ_B ? P * BJ_B + c : Qb * BJ_B + (c - BJ_B);
}

// Partial Grams over the `rows` rows (a multiple of 64; at most BJ_MAXCH
// chunks cover Dp) of chunk blockIdx.y for block pair blockIdx.x:
// part[(k nchunk + c)][tile][i][j], tiles X_P^T X_P, X_P^T X_Q, X_Q^T X_Q.
// FP64 MFMA 16x16x4: lane (col, kq) holds rows row0 + 4 kq + u (u < 4) of
// column col of each block (one 32-byte load each), and the k index of step
// u is the row row0 + 4 kq + u for both operands.
__global__ __launch_bounds__(256) void bj_gram_kernel(
    const double *__restrict__ A, int Dp, int nb, int t, int nchunk, int rows,
    double *__restrict__ part) {
  __shared__ double red[4][3][256];
  const int k = blockIdx.x, c = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  int P, Qb;
  bj_pair(nb, t, k, P, Qb);
  const double *xp = A + (int64_t)(P * BJ_B + col) * Dp + 4 * kq;
  const double *xq = A + (int64_t)(Qb * BJ_B + col) * Dp + 4 * kq;
  d4 gpp = {0.0, 0.0, 0.0, 0.0}, gpq = gpp, gqq = gpp;
  const int per_wave = rows / 4;  // a multiple of 16
  const int rbeg = c * rows + wave * per_wave;
#pragma unroll 4
  for (int g = 0; g < per_wave / 16; ++g) {
    const int row0 = rbeg + 16 * g;
    if (row0 >= Dp) break;
    const d4 a = *(const d4 *)(xp + row0);
    const d4 b = *(const d4 *)(xq + row0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      gpp = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], a[u], gpp, 0, 0, 0);
      gpq = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], gpq, 0, 0, 0);
      gqq = __builtin_amdgcn_mfma_f64_16x16x4f64(b[u], b[u], gqq, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = (kq + 4 * r) * 16 + col;
    red[wave][0][e] = gpp[r];
    red[wave][1][e] = gpq[r];
    red[wave][2][e] = gqq[r];
  }
  __syncthreads();
  double *out = part + ((int64_t)k * nchunk + c) * 768;
  for (int e = threadIdx.x; e < 768; e += 256) {
    const int tile = e >> 8, idx = e & 255;
    out[e] = (red[0][tile][idx] + red[1][tile][idx]) +
             (red[2][tile][idx] + red[3][tile][idx]);
  }
}

__device__ inline void bj_pair32(int r, int kk, int &p, int &q) {
  if (kk == 0) {
    p = r % 31;
    q = 31;
  } else {
    p = (r + kk) % 31;
    q = (r - kk + 31) % 31;
  }
}

// One workgroup per block pair: sums the partial Grams, and if any column
// pair fails the orthogonality test, applies one cyclic sweep of two-sided
// Jacobi to G accumulating U; else marks the pair skipped.  (One sweep per
// visit of the block pair is cheaper overall than diagonalising G fully:
// the outer sweeps revisit every pair anyway.)  A round applies 16
// disjoint rotations J (pair (p, q): column p' = c p - s q, q' = s p + c q);
// G' = J^T G J maps each 2 x 2 block (rows of pair a, columns of pair b)
// from its own four entries, so thread a * 16 + b updates one block in
// place and the rotated pair's off-diagonal is set to zero.  Counts the
// block pairs rotated.
__global__ __launch_bounds__(256) void bj_eig_kernel(
    const double *__restrict__ part, int nchunk, double tol,
    double *__restrict__ Uout, int *__restrict__ skip, int *__restrict__ cnt) {
  __shared__ double G[BJ_W][BJ_W + 1];
  __shared__ double U[BJ_W][BJ_W + 1];
  __shared__ double cs[16][2];
  __shared__ int need;
  const int k = blockIdx.x, tid = threadIdx.x;
  const double *pk = part + (int64_t)k * nchunk * 768;
  if (tid == 0) need = 0;
  for (int e = tid; e < 768; e += 256) {
    // every chunk's partial in flight at once (nchunk <= BJ_MAXCH; addresses
    // clamped), then added in chunk order
    double v[BJ_MAXCH];
#pragma unroll
    for (int c = 0; c < BJ_MAXCH; ++c)
      v[c] = pk[(int64_t)min(c, nchunk - 1) * 768 + e];
    double sum = 0.0;
#pragma unroll
    for (int c = 0; c < BJ_MAXCH; ++c)
      if (c < nchunk) sum += v[c];
    const int tile = e >> 8, i = (e & 255) >> 4, j = e & 15;
    if (tile == 0) {
      G[i][j] = sum;
    } else if (tile == 1) {
      G[i][BJ_B + j] = sum;
      G[BJ_B + j][i] = sum;
    } else {
      G[BJ_B + i][BJ_B + j] = sum;
    }
  }
  for (int e = tid; e < BJ_W * BJ_W; e += 256)
    U[e >> 5][e & 31] = (e >> 5) == (e & 31) ? 1.0 : 0.0;
  __syncthreads();
  for (int e = tid; e < BJ_W * BJ_W; e += 256) {
    const int i = e >> 5, j = e & 31;
    if (i < j && G[i][j] * G[i][j] > tol * tol * (G[i][i] * G[j][j])) need = 1;
  }
  __syncthreads();
  if (!need) {
    if (tid == 0) skip[k] = 1;
    return;
  }
  const int ka = tid >> 4, kb = tid & 15;  // this thread's 2 x 2 block of G
  {
    for (int r = 0; r < 31; ++r) {
      if (tid < 16) {
        int p, q;
        bj_pair32(r, tid, p, q);
        const double al = G[p][p], be = G[q][q], ga = G[p][q];
        double c = 1.0, s = 0.0;
        if (ga * ga > tol * tol * (al * be)) {
          // the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = d / (2 ga),
          // as sign(d) 2 ga / (|d| + sqrt(d^2 + 4 ga^2)): one square root
          // and one division
          const double d = be - al;
          const double tt = (d >= 0.0 ? 2.0 * ga : -2.0 * ga) /
                            (fabs(d) + sqrt(d * d + 4.0 * ga * ga));
          c = rsqrt(1.0 + tt * tt);
          s = c * tt;
        }
        cs[tid][0] = c;
        cs[tid][1] = s;
      }
      __syncthreads();
      {
        const double ca = cs[ka][0], sa = cs[ka][1];
        const double cb = cs[kb][0], sb = cs[kb][1];
        if (sa != 0.0 || sb != 0.0) {
          int p, q, u, v;
          bj_pair32(r, ka, p, q);
          bj_pair32(r, kb, u, v);
          const double gpu = G[p][u], gpv = G[p][v], gqu = G[q][u], gqv = G[q][v];
          // columns: (u, v) -> (cb u - sb v, sb u + cb v)
          const double hpu = cb * gpu - sb * gpv, hpv = sb * gpu + cb * gpv;
          const double hqu = cb * gqu - sb * gqv, hqv = sb * gqu + cb * gqv;
          // rows: (p, q) -> (ca p - sa q, sa p + ca q)
          G[p][u] = ca * hpu - sa * hqu;
          G[q][u] = sa * hpu + ca * hqu;
          G[p][v] = ca * hpv - sa * hqv;
          G[q][v] = sa * hpv + ca * hqv;
          if (ka == kb && sa != 0.0) {
            G[p][v] = 0.0;
            G[q][u] = 0.0;
          }
        }
      }
      for (int e = tid; e < BJ_W * 16; e += 256) {
        const int i = e >> 4, kk = e & 15;
        const double s = cs[kk][1];
        if (s != 0.0) {
          const double c = cs[kk][0];
          int p, q;
          bj_pair32(r, kk, p, q);
          const double x = U[i][p], y = U[i][q];
          U[i][p] = c * x - s * y;
          U[i][q] = s * x + c * y;
        }
      }
      __syncthreads();
    }
  }
  double *uo = Uout + (int64_t)k * BJ_W * BJ_W;
  for (int e = tid; e < BJ_W * BJ_W; e += 256) uo[e] = U[e >> 5][e & 31];
  if (tid == 0) {
    skip[k] = 0;
    atomicAdd(cnt, 1);
  }
}

// X <- X U for the 32 columns of block pair blockIdx.x, in A and in V, over
// the rows of chunk blockIdx.y (in place: each wave loads its 16-row group
// of all 32 columns before writing it back).  Computed as Y^T = U^T X^T so
// that a lane's outputs run down a column: A operand U[4 s + kq][16 it +
// col], B operand X[row0 + col][position 4 s + kq], output lane r holds
// Y[row0 + col][position 16 it + kq + 4 r].
__global__ __launch_bounds__(256) void bj_rotate_kernel(
    double *A, double *V, int Dp, int nb, int t,
    const double *__restrict__ Uall, const int *__restrict__ skip) {
  const int k = blockIdx.x, c = blockIdx.y;
  if (skip[k]) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  int P, Qb;
  bj_pair(nb, t, k, P, Qb);
  const double *Uk = Uall + (int64_t)k * BJ_W * BJ_W;
  double ua[2][8];
#pragma unroll
  for (int it = 0; it < 2; ++it)
#pragma unroll
    for (int s = 0; s < 8; ++s) ua[it][s] = Uk[(4 * s + kq) * BJ_W + 16 * it + col];
  int64_t cin[8], cout0[4], cout1[4];
#pragma unroll
  for (int s = 0; s < 8; ++s) cin[s] = (int64_t)bj_col(P, Qb, 4 * s + kq) * Dp;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cout0[r] = (int64_t)bj_col(P, Qb, kq + 4 * r) * Dp;
    cout1[r] = (int64_t)bj_col(P, Qb, BJ_B + kq + 4 * r) * Dp;
  }
  const int rbeg = c * BJ_CH + wave * 64;
#pragma unroll
  for (int mat = 0; mat < 2; ++mat) {
    double *X = mat ? V : A;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int row0 = rbeg + 16 * g;
      if (row0 >= Dp) break;
      double xb[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) xb[s] = X[cin[s] + row0 + col];
      d4 y0 = {0.0, 0.0, 0.0, 0.0}, y1 = y0;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        y0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[0][s], xb[s], y0, 0, 0, 0);
        y1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ua[1][s], xb[s], y1, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        X[cout0[r] + row0 + col] = y0[r];
        X[cout1[r] + row0 + col] = y1[r];
      }
    }
  }
}

// Column k after convergence: a_k = (H + sigma I) v_k.  Eigenvalue by the
// Rayleigh quotient a_k.v_k / v_k.v_k - sigma (second order in the
// eigenvector's error, unlike the norm |a_k|); amplitudes w_ik from the
// normalised v_k.
__global__ void inner_extract_kernel(const double *A, const double *V, int n,
                                     int N, int Dp, double sigma, double a,
                                     double *lam, double *w) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int D = n * N;
  if (k >= D) return;
  const double *ak = A + (int64_t)k * Dp, *vk = V + (int64_t)k * Dp;
  double av = 0.0, vv = 0.0;
  for (int r = 0; r < D; ++r) {
    av = fma(ak[r], vk[r], av);
    vv = fma(vk[r], vk[r], vv);
  }
  lam[k] = av / vv - sigma;
  const double f = sqrt(2.0) * sqrt(2.0 / a) / sqrt(vv);
  for (int i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int m = 0; m < N; ++m) acc += (m & 1 ? -1.0 : 1.0) * vk[i * N + m];
    w[(int64_t)i * D + k] = f * acc;
  }
}

// Gauss-Legendre nodes r and weights w on [0, a].  Each zero x = -cos(th)
// of P_Q (th in (0, pi/2], the mirror x = cos(th) for the upper half) comes
// from Newton's method in th on the three-term recurrence, in long double
// so that th is exact to double rounding; r = a sin^2(th/2) (a cos^2(th/2)
// mirrored) keeps the full relative accuracy of the nodes next to r = 0,
// where the centrifugal term grows as 1/r^2, and the weight
// a / ((1 - x^2) P_Q'(x)^2) uses 1 - x^2 = sin^2(th).
static void gauss_legendre(int Q, double a, std::vector<double> &r,
                           std::vector<double> &w) {
  typedef long double ld;
  const ld pi = 3.141592653589793238462643383279502884L;
  r.assign(Q, 0.0);
  w.assign(Q, 0.0);
  auto recur = [Q](ld x, ld &pq, ld &pm) {
    ld p0 = 1.0L, p1 = x;
    for (int k = 2; k <= Q; ++k) {
      const ld pk = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    pq = Q == 1 ? x : p1;
    pm = Q == 1 ? 1.0L : p0;
  };
  const int h = (Q + 1) / 2;
  for (int i = 0; i < h; ++i) {
    ld th = pi * (i + 0.75L) / (Q + 0.5L), pq, pm;
    for (int it = 0; it < 12; ++it) {
      recur(cosl(th), pq, pm);
      const ld step = pq * sinl(th) / (Q * (cosl(th) * pq - pm));
      th -= step;
      if (fabsl(step) <= 1e-17L * th) {  // one more polishing step
        recur(cosl(th), pq, pm);
        th -= pq * sinl(th) / (Q * (cosl(th) * pq - pm));
        break;
      }
    }
    const ld x = cosl(th), s = sinl(th);
    recur(x, pq, pm);
    const ld d = Q * (x * pq - pm);
    const ld wt = (ld)a * s * s / (d * d);
    const ld sh = sinl(th / 2), ch = cosl(th / 2);
    r[i] = (double)((ld)a * sh * sh);
    w[i] = (double)wt;
    if (i < Q - h) {
      r[Q - 1 - i] = (double)((ld)a * ch * ch);
      w[Q - 1 - i] = (double)wt;
    }
  }
}

}  // namespace rmx

using namespace rmx;

extern "C" {

int rm_inner_region(const rm_inner_desc *d, double *E_pole, double *w,
                    int32_t *sweeps, int64_t *rotations, void *stream) {
  const char *fn = "rm_inner_region";
  if (!d || !E_pole || !w) return in_fail(RM_ERR_ARG, std::string(fn) + ": null pointer");
  const int n = d->n_chan, N = d->n_basis;
  if (n < 1 || N < 1) return in_fail(RM_ERR_ARG, std::string(fn) + ": n_chan < 1 or n_basis < 1");
  if ((int64_t)n * N > BJ_DMAX)
    return in_fail(RM_ERR_ARG, std::string(fn) + ": n_chan * n_basis > 16384");
  if (!(d->a > 0.0) || !std::isfinite(d->a) || !(d->z >= 0.0) || !std::isfinite(d->z))
    return in_fail(RM_ERR_ARG, std::string(fn) + ": a must be > 0 and z >= 0");
  if (!d->e_thr || !d->l || !d->depth || !d->range)
    return in_fail(RM_ERR_ARG, std::string(fn) + ": null model array");
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(d->e_thr[i]) || d->l[i] < 0 || d->l[i] > 12)
      return in_fail(RM_ERR_ARG, std::string(fn) + ": bad threshold or l");
    for (int j = 0; j < n; ++j) {
      const double dd = d->depth[i * n + j], rr = d->range[i * n + j];
      if (!std::isfinite(dd) || !(rr > 0.0) || !std::isfinite(rr) ||
          dd != d->depth[j * n + i] || rr != d->range[j * n + i])
        return in_fail(RM_ERR_ARG, std::string(fn) + ": depth/range not finite, positive and symmetric");
    }
  }
  const int Q = d->n_quad > 0 ? d->n_quad : N + 48;
  if (Q > 16384) return in_fail(RM_ERR_ARG, std::string(fn) + ": n_quad > 16384");
  if ((double)n * n * (Q + 3) * 8.0 > 8.0e9)
    return in_fail(RM_ERR_ARG, std::string(fn) + ": quadrature table n_chan^2 n_quad over 8 GB");
  hipStream_t st = (hipStream_t)stream;
  const int D = n * N, Dp = (D + BJ_W - 1) / BJ_W * BJ_W;  // even block count
  const int nb = Dp / BJ_B, npair = nb / 2, nchunk = (Dp + BJ_CH - 1) / BJ_CH;
  // Gram chunks: 64-row multiples, at most BJ_MAXCH of them (the eigen
  // kernel loads every chunk's partial at once)
  const int gram_rows = 64 * ((Dp + 64 * BJ_MAXCH - 1) / (64 * BJ_MAXCH));
  const int gchunk = (Dp + gram_rows - 1) / gram_rows;
  std::vector<double> rq, wq;
  gauss_legendre(Q, d->a, rq, wq);
  // device: A, V [Dp][Dp]; rq, wq [Q]; model arrays; lam [D]; w [n][D];
  // Gershgorin bounds [D]; quadrature tables; partial Grams [npair][nchunk]
  // [3][16][16]; rotations [npair][32][32]; l [n]; skip flags [npair];
  // block-pair counter
  const size_t nsq = (size_t)Dp * Dp;
  const size_t npart = (size_t)npair * gchunk * 768, nu = (size_t)npair * BJ_W * BJ_W;
  const int Qp = (Q + 3) / 4 * 4;
  const size_t ndbl = 2 * nsq + 2 * (size_t)Q + (size_t)n + 2 * (size_t)n * n +
                      (size_t)D + (size_t)n * D + (size_t)D + (size_t)N * Qp +
                      (size_t)n * n * Qp + npart + nu;
  char *ws = nullptr;
  const size_t bytes = ndbl * sizeof(double) +
                       ((size_t)n + (size_t)npair) * sizeof(int32_t) + 64;
  hipError_t e = hipMalloc((void **)&ws, bytes);
  if (e != hipSuccess)
    return in_fail(e == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP,
                   std::string(fn) + ": " + hipGetErrorString(e));
  double *A = (double *)ws, *V = A + nsq, *drq = V + nsq, *dwq = drq + Q;
  double *de = dwq + Q, *ddep = de + n, *dran = ddep + (size_t)n * n;
  double *lam = dran + (size_t)n * n, *dw = lam + D, *lb = dw + (size_t)n * D;
  double *phi = lb + D, *wv = phi + (size_t)N * Qp;
  double *part = wv + (size_t)n * n * Qp, *Ub = part + npart;
  int32_t *dl = (int32_t *)(Ub + nu);
  int *skip = (int *)(dl + n);
  int *cnt = (int *)(((uintptr_t)(skip + npair) + 15) & ~(uintptr_t)15);
  int used = 0;
  bool converged = false;
  int64_t rot_total = 0;
  std::vector<double> hlb(D), hlam(D), hw((size_t)n * D);
  auto hip_ok = [&](hipError_t x) { if (e == hipSuccess) e = x; return e == hipSuccess; };
  hip_ok(hipMemcpyAsync(drq, rq.data(), Q * sizeof(double), hipMemcpyHostToDevice, st));
  hip_ok(hipMemcpyAsync(dwq, wq.data(), Q * sizeof(double), hipMemcpyHostToDevice, st));
  hip_ok(hipMemcpyAsync(de, d->e_thr, n * sizeof(double), hipMemcpyHostToDevice, st));
  hip_ok(hipMemcpyAsync(ddep, d->depth, (size_t)n * n * sizeof(double), hipMemcpyHostToDevice, st));
  hip_ok(hipMemcpyAsync(dran, d->range, (size_t)n * n * sizeof(double), hipMemcpyHostToDevice, st));
  hip_ok(hipMemcpyAsync(dl, d->l, n * sizeof(int32_t), hipMemcpyHostToDevice, st));
  ProfileScope *asm_scope = new ProfileScope(9, st);
  if (e == hipSuccess) {
    const int64_t nt = (int64_t)N * Qp + (int64_t)n * n * Qp;
    hipLaunchKernelGGL(inner_tables_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256),
                       0, st, n, N, Q, Qp, d->a, d->z, drq, dwq, de, dl, ddep, dran, phi, wv);
    hip_ok(hipGetLastError());
  }
  if (e == hipSuccess) {
    const unsigned nt32 = (unsigned)((N + 31) / 32);
    hipLaunchKernelGGL(inner_assemble_kernel, dim3((unsigned)(n * n), nt32, nt32), dim3(64),
                       0, st, n, N, Qp, d->a, phi, wv, A, Dp);
    hip_ok(hipGetLastError());
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(inner_gershgorin_kernel, dim3((unsigned)((D + 255) / 256)),
                       dim3(256), 0, st, A, D, Dp, lb);
    hip_ok(hipGetLastError());
  }
  delete asm_scope;
  hip_ok(hipMemcpyAsync(hlb.data(), lb, D * sizeof(double), hipMemcpyDeviceToHost, st));
  hip_ok(hipStreamSynchronize(st));
  double sigma = 0.0;
  if (e == hipSuccess) {
    const double mn = *std::min_element(hlb.begin(), hlb.end());
    sigma = std::max(0.0, -mn) + 1.0;  // H + sigma I has eigenvalues >= 1
    hipLaunchKernelGGL(inner_init_kernel, dim3((unsigned)((nsq + 255) / 256)), dim3(256),
                       0, st, A, V, D, Dp, sigma);
    hip_ok(hipGetLastError());
  }
  // sweeps until no pair needs a rotation
  const int max_sweeps = 40;
  // LAPACK's one-sided Jacobi stops at sqrt(m) eps; a few times that covers
  // the rounding of the Gram entries
  const double tol = 8.0 * std::sqrt((double)Dp) * 2.220446049250313e-16;
  for (int sw = 0; sw < max_sweeps && e == hipSuccess; ++sw) {
    int h_cnt = 0;
    hip_ok(hipMemsetAsync(cnt, 0, sizeof(int), st));
    {
      ProfileScope scope(8, st);
      for (int t = 0; t < nb - 1 && e == hipSuccess; ++t) {
        hipLaunchKernelGGL(bj_gram_kernel, dim3(npair, gchunk), dim3(256), 0, st, A, Dp,
                           nb, t, gchunk, gram_rows, part);
        hipLaunchKernelGGL(bj_eig_kernel, dim3(npair), dim3(256), 0, st, part, gchunk,
                           tol, Ub, skip, cnt);
        hipLaunchKernelGGL(bj_rotate_kernel, dim3(npair, nchunk), dim3(256), 0, st, A, V,
                           Dp, nb, t, Ub, skip);
        hip_ok(hipGetLastError());
      }
    }
    hip_ok(hipMemcpyAsync(&h_cnt, cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    hip_ok(hipStreamSynchronize(st));
    used = sw + 1;
    rot_total += h_cnt;
    if (h_cnt == 0) {
      converged = true;
      break;
    }
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(inner_extract_kernel, dim3((unsigned)((D + 255) / 256)), dim3(256),
                       0, st, A, V, n, N, Dp, sigma, d->a, lam, dw);
    hip_ok(hipGetLastError());
  }
  hip_ok(hipMemcpyAsync(hlam.data(), lam, D * sizeof(double), hipMemcpyDeviceToHost, st));
  hip_ok(hipMemcpyAsync(hw.data(), dw, (size_t)n * D * sizeof(double), hipMemcpyDeviceToHost, st));
  hip_ok(hipStreamSynchronize(st));
  (void)hipFree(ws);
  if (e != hipSuccess)
    return in_fail(e == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP,
                   std::string(fn) + ": " + hipGetErrorString(e));
  // ascending poles, amplitudes permuted with them
  std::vector<int> ord(D);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return hlam[x] < hlam[y]; });
  for (int k = 0; k < D; ++k) {
    E_pole[k] = hlam[ord[k]];
    for (int i = 0; i < n; ++i) w[(size_t)i * D + k] = hw[(size_t)i * D + ord[k]];
  }
  if (sweeps) *sweeps = used;
  if (rotations) *rotations = rot_total;
  if (!converged) return in_fail(RM_ERR_NUMERIC, std::string(fn) + ": Jacobi did not converge in 40 sweeps");
  return RM_OK;
}

// Several model Hamiltonians at once: each solve runs on a stream of its
// own, driven by one of up to 8 host threads (a solve waits on its stream
// once per sweep), so the small solves' kernels overlap on the device.
int rm_inner_region_batch(const rm_inner_desc *descs, int32_t count,
                          double *const *E_pole, double *const *w,
                          int32_t *sweeps, int64_t *rotations, void *stream) {
  const char *fn = "rm_inner_region_batch";
  if (count < 0) return in_fail(RM_ERR_ARG, std::string(fn) + ": count < 0");
  if (count == 0) return RM_OK;
  if (!descs || !E_pole || !w) return in_fail(RM_ERR_ARG, std::string(fn) + ": null pointer");
  for (int b = 0; b < count; ++b)
    if (!E_pole[b] || !w[b])
      return in_fail(RM_ERR_ARG, std::string(fn) + ": null output of item " + std::to_string(b));
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  // the caller's stream first: work already queued there precedes the solves
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return in_fail(RM_ERR_HIP, std::string(fn) + ": " + hipGetErrorString(e));
  std::vector<int> codes(count, RM_OK);
  std::vector<std::string> msgs(count);
  std::atomic<int> next(0);
  auto worker = [&]() {
    if (hipSetDevice(dev) != hipSuccess) return;
    hipStream_t st = nullptr;
    const bool own = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (int b = next++; b < count; b = next++) {
      if (!own) {
        codes[b] = RM_ERR_HIP;
        msgs[b] = "stream creation failed";
        continue;
      }
      codes[b] = rm_inner_region(&descs[b], E_pole[b], w[b],
                                 sweeps ? &sweeps[b] : nullptr,
                                 rotations ? &rotations[b] : nullptr, st);
      if (codes[b] != RM_OK) msgs[b] = rm_last_error();
    }
    if (own) (void)hipStreamDestroy(st);
  };
  const int nt = std::min<int>(count, 8);
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t) pool.emplace_back(worker);
  for (auto &t : pool) t.join();
  if (next.load() < count) return in_fail(RM_ERR_HIP, std::string(fn) + ": hipSetDevice failed");
  for (int b = 0; b < count; ++b)
    if (codes[b] != RM_OK)
      return in_fail(codes[b], std::string(fn) + ": item " + std::to_string(b) + ": " + msgs[b]);
  return RM_OK;
}

}  // extern "C"
