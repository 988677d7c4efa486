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
// then column k is (H + sigma I) v_k with v_k an eigenvector.  In each
// round-robin step every column pair is orthogonalised by one wavefront.  w_ik = sqrt2 sum_m
// V_(i,m),k phi_m(a) with phi_m(a) = sqrt(2/a) (-1)^m, the convention of
// R = (1/2a) sum_k w_ik w_jk / (E_k - E).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "rm_internal.h"

namespace rmx {

const char *set_error(int code, const char *msg);  // defined in rm_api.hip

static int in_fail(int code, const std::string &msg) {
  set_error(code, msg.c_str());
  return code;
}

// Tables of the quadrature: phi[m][q] = sqrt(2/a) sin(kappa_m r_q) and
// wv[i][j][q] = w_q W_ij(r_q) (W without E).
__global__ void inner_tables_kernel(int n, int N, int Q, double a, double z,
                                    const double *__restrict__ rq,
                                    const double *__restrict__ wq,
                                    const double *__restrict__ e_thr,
                                    const int32_t *__restrict__ l,
                                    const double *__restrict__ depth,
                                    const double *__restrict__ range,
                                    double *__restrict__ phi,
                                    double *__restrict__ wv) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nphi = (int64_t)N * Q, nw = (int64_t)n * n * Q;
  if (idx < nphi) {
    const int m = (int)(idx / Q), q = (int)(idx % Q);
    phi[idx] = sqrt(2.0 / a) * sin((m + 0.5) * M_PI / a * rq[q]);
  } else if (idx < nphi + nw) {
    const int64_t t = idx - nphi;
    const int ij = (int)(t / Q), q = (int)(t % Q);
    const int i = ij / n, j = ij % n;
    const double r = rq[q], x = r / range[ij];
    double v = -depth[ij] * exp(-x * x);
    if (i == j) v += l[i] * (l[i] + 1.0) / (r * r) - 2.0 * z / r + e_thr[i];
    wv[t] = wq[q] * v;
  }
}

// H[p][p'] (column-major, leading dimension ld) for p = i N + m:
// kappa_m^2 delta + sum_q phi_m(r_q) w_q W_ij(r_q) phi_m'(r_q).
__global__ void inner_assemble_kernel(int n, int N, int Q, double a,
                                      const double *__restrict__ phi,
                                      const double *__restrict__ wv,
                                      double *__restrict__ H, int ld) {
  const int64_t D = (int64_t)n * N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= D * D) return;
  const int64_t col = idx / D, row = idx % D;
  if (row < col) return;  // lower triangle, mirrored below
  const int i = (int)(row / N), m = (int)(row % N);
  const int j = (int)(col / N), mp = (int)(col % N);
  const double *pm = phi + (int64_t)m * Q, *pp = phi + (int64_t)mp * Q;
  const double *w = wv + (int64_t)(i * n + j) * Q;
  double acc = 0.0;
  for (int q = 0; q < Q; ++q) acc = fma(pm[q] * pp[q], w[q], acc);
  if (row == col) {
    const double km = (m + 0.5) * M_PI / a;
    acc += km * km;
  }
  H[col * ld + row] = acc;
  H[row * ld + col] = acc;
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

// A = H + sigma I on the first D columns; padding column (if any) zero; V = I.
__global__ void inner_init_kernel(double *A, double *V, int D, int Dp,
                                  double sigma) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)Dp * Dp) return;
  const int64_t c = idx / Dp, r = idx % Dp;
  if (c >= D || r >= D) A[idx] = 0.0;
  else if (r == c) A[idx] += sigma;
  V[idx] = (r == c) ? 1.0 : 0.0;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One round-robin step t of a sweep over Dp (even) columns: pair k of the
// circle method ((t, Dp - 1) for k = 0, else (t + k, t - k) mod (Dp - 1))
// is orthogonalised by wavefront k.  Counts the rotations done.
__global__ __launch_bounds__(256) void inner_jacobi_step_kernel(
    double *A, double *V, int Dp, int t, double tol, int *rot_count) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= Dp / 2) return;
  const int L = Dp - 1;
  int p, q;
  if (k == 0) {
    p = t % L;
    q = L;
  } else {
    p = (t + k) % L;
    q = (t - k + L) % L;
  }
  double *ap = A + (int64_t)p * Dp, *aq = A + (int64_t)q * Dp;
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int r = lane; r < Dp; r += 64) {
    const double x = ap[r], y = aq[r];
    al = fma(x, x, al);
    be = fma(y, y, be);
    ga = fma(x, y, ga);
  }
  al = wave_sum(al);
  be = wave_sum(be);
  ga = wave_sum(ga);
  if (!(fabs(ga) > tol * sqrt(al * be))) return;  // already orthogonal
  // rotation zeroing the off-diagonal of [[al, ga], [ga, be]]
  const double ze = (be - al) / (2.0 * ga);
  const double tt = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
  const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
  for (int r = lane; r < Dp; r += 64) {
    const double x = ap[r], y = aq[r];
    ap[r] = c * x - s * y;
    aq[r] = s * x + c * y;
  }
  double *vp = V + (int64_t)p * Dp, *vq = V + (int64_t)q * Dp;
  for (int r = lane; r < Dp; r += 64) {
    const double x = vp[r], y = vq[r];
    vp[r] = c * x - s * y;
    vq[r] = s * x + c * y;
  }
  if (lane == 0) atomicAdd(rot_count, 1);
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
  if ((int64_t)n * N > 4096)
    return in_fail(RM_ERR_ARG, std::string(fn) + ": n_chan * n_basis > 4096");
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
  hipStream_t st = (hipStream_t)stream;
  const int D = n * N, Dp = D + (D & 1);
  std::vector<double> rq, wq;
  gauss_legendre(Q, d->a, rq, wq);
  // device: A, V [Dp][Dp]; rq, wq [Q]; model arrays; lam [D]; w [n][D];
  // Gershgorin bounds [D]; rotation counter
  const size_t nsq = (size_t)Dp * Dp;
  const size_t ndbl = 2 * nsq + 2 * (size_t)Q + (size_t)n + 2 * (size_t)n * n +
                      (size_t)D + (size_t)n * D + (size_t)D + (size_t)N * Q +
                      (size_t)n * n * Q;
  char *ws = nullptr;
  const size_t bytes = ndbl * sizeof(double) + (size_t)n * sizeof(int32_t) + 64;
  hipError_t e = hipMalloc((void **)&ws, bytes);
  if (e != hipSuccess)
    return in_fail(e == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP,
                   std::string(fn) + ": " + hipGetErrorString(e));
  double *A = (double *)ws, *V = A + nsq, *drq = V + nsq, *dwq = drq + Q;
  double *de = dwq + Q, *ddep = de + n, *dran = ddep + (size_t)n * n;
  double *lam = dran + (size_t)n * n, *dw = lam + D, *lb = dw + (size_t)n * D;
  double *phi = lb + D, *wv = phi + (size_t)N * Q;
  int32_t *dl = (int32_t *)(wv + (size_t)n * n * Q);
  int *cnt = (int *)(((uintptr_t)(dl + n) + 15) & ~(uintptr_t)15);
  int used = 0;
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
    const int64_t nt = (int64_t)N * Q + (int64_t)n * n * Q;
    hipLaunchKernelGGL(inner_tables_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256),
                       0, st, n, N, Q, d->a, d->z, drq, dwq, de, dl, ddep, dran, phi, wv);
    hip_ok(hipGetLastError());
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(inner_assemble_kernel,
                       dim3((unsigned)(((int64_t)D * D + 255) / 256)), dim3(256), 0, st,
                       n, N, Q, d->a, phi, wv, A, Dp);
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
  // the rounding of the wavefront's dot products
  const double tol = 8.0 * std::sqrt((double)Dp) * 2.220446049250313e-16;
  for (int sw = 0; sw < max_sweeps && e == hipSuccess; ++sw) {
    int h_cnt = 0;
    hip_ok(hipMemsetAsync(cnt, 0, sizeof(int), st));
    {
      ProfileScope scope(8, st);
      for (int t = 0; t < Dp - 1 && e == hipSuccess; ++t) {
        hipLaunchKernelGGL(inner_jacobi_step_kernel, dim3((unsigned)((Dp / 2 + 3) / 4)),
                           dim3(256), 0, st, A, V, Dp, t, tol, cnt);
        hip_ok(hipGetLastError());
      }
    }
    hip_ok(hipMemcpyAsync(&h_cnt, cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    hip_ok(hipStreamSynchronize(st));
    used = sw + 1;
    rot_total += h_cnt;
    if (h_cnt == 0) break;
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
  if (used >= max_sweeps) return in_fail(RM_ERR_NUMERIC, std::string(fn) + ": Jacobi did not converge in 40 sweeps");
  return RM_OK;
}

}  // extern "C"
