// Learned adaptive mesh: a small MLP trained on the device, and the
// density -> mesh placement.
//
// The network maps per-window features of a scattering system to a
// log-density of mesh points.  Layers are dense, width W, SiLU activations
// (x sigma(x)) between them and a linear output.  Matrix products run on the
// gfx950 matrix cores with BF16 operands (weights and activations rounded to
// BF16 when staged in LDS) and FP32 accumulation (v_mfma_f32_16x16x32_bf16);
// a debug precision runs the same kernels with FP32 operands
// (v_mfma_f32_16x16x4f32).  Master weights, gradients and Adam moments are
// FP32.  Parameters are one flat FP32 array: per layer W_l [out][in] then
// b_l [out].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rmatrix.h"

namespace rmx {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

const char *set_error(int code, const char *msg);  // defined in rm_api.hip

constexpr int GT = 64;   // output tile edge
constexpr int GK = 32;   // k chunk

// C[i][j] (ldc) = sum_k A(i,k) B(k,j) + (accumulate ? C : 0)
// A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj], FP32 in memory.
template <bool BF16>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(
    const float *A, int64_t sai, int64_t sak, const float *B, int64_t sbk,
    int64_t sbj, float *C, int ldc, int M, int N, int K, int accumulate) {
  __shared__ float Af[BF16 ? 1 : GT][GK + 1];
  __shared__ float Bf[BF16 ? 1 : GT][GK + 1];
  __shared__ __bf16 Ab[BF16 ? GT : 1][GK + 8];
  __shared__ __bf16 Bb[BF16 ? GT : 1][GK + 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const int col = lane & 15, kq = lane >> 4;
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int q = tid; q < GT * GK; q += 256) {
      const int r = q / GK, k = q % GK;
      const int gi = i0 + r, gj = j0 + r, gk = k0 + k;
      const float av = (gi < M && gk < K) ? A[gi * sai + gk * sak] : 0.f;
      const float bv = (gj < N && gk < K) ? B[gk * sbk + gj * sbj] : 0.f;
      if (BF16) {
        Ab[r][k] = (__bf16)av;
        Bb[r][k] = (__bf16)bv;
      } else {
        Af[r][k] = av;
        Bf[r][k] = bv;
      }
    }
    __syncthreads();
    if (BF16) {
      bf8 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = *(const bf8 *)&Ab[wi + 16 * t + col][8 * kq];
        b[t] = *(const bf8 *)&Bb[wj + 16 * t + col][8 * kq];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y],
                                                              acc[x][y], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < GK; kk += 4) {
        float a[2], b[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          a[t] = Af[wi + 16 * t + col][kk + kq];
          b[t] = Bf[wj + 16 * t + col][kk + kq];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y],
                                                             acc[x][y], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // D[i][j]: j = lane%16, i = 4*(lane/16) + r
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wi + 16 * x + 4 * kq + r;
        const int gj = j0 + wj + 16 * y + col;
        if (gi < M && gj < N) {
          float *c = C + (int64_t)gi * ldc + gj;
          *c = (accumulate ? *c : 0.f) + acc[x][y][r];
        }
      }
}

__device__ inline float sigm(float x) { return 1.f / (1.f + expf(-x)); }

// Z[b][j] += bias[j]; A = silu(Z) (act) or copy
__global__ void bias_act_kernel(float *Z, float *A, const float *bias, int B,
                                int N, int act) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * N) return;
  const float z = Z[idx] + bias[idx % N];
  Z[idx] = z;
  A[idx] = act ? z * sigm(z) : z;
}

// dZ = dA * silu'(Z)
__global__ void act_bwd_kernel(const float *dA, const float *Z, float *dZ,
                               int64_t count) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= count) return;
  const float z = Z[idx];
  const float s = sigm(z);
  dZ[idx] = dA[idx] * s * (1.f + z * (1.f - s));
}

// db[j] = sum_b dZ[b][j]
__global__ void bias_grad_kernel(const float *dZ, float *db, int B, int N) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * N + j];
  db[j] = s;
}

// MSE: loss = mean (y - t)^2, dY = 2 (y - t) / B; one workgroup
__global__ void mse_kernel(const float *Y, const float *T, float *dY,
                           float *loss, int B) {
  __shared__ float red[256];
  float s = 0.f;
  for (int b = threadIdx.x; b < B; b += 256) {
    const float d = Y[b] - T[b];
    dY[b] = 2.f * d / B;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / B;
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v,
                            int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void copy_f32_kernel(const float *s, float *d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// Mesh placement: cum[w] = exclusive prefix of the floored, normalised
// density; one workgroup, sequential blocks of windows per thread.
__global__ void density_cdf_kernel(const float *dens, int nw, double floor_frac,
                                   double *cum) {
  __shared__ double part[256];
  __shared__ double tot_s;
  const int tid = threadIdx.x;
  const int per = (nw + 255) / 256;
  const int w0 = min(nw, tid * per), w1 = min(nw, w0 + per);
  double s = 0.0;
  for (int w = w0; w < w1; ++w) s += fmax((double)dens[w], 0.0);
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int q = 0; q < 256; ++q) {
      const double v = part[q];
      part[q] = t;
      t += v;
    }
    tot_s = t;
  }
  __syncthreads();
  const double tot = tot_s;
  const double fl = floor_frac / nw;
  const double sc = tot > 0.0 ? (1.0 - floor_frac) / tot : 0.0;
  const double fl2 = tot > 0.0 ? fl : 1.0 / nw;
  double run = part[tid] * sc + w0 * fl2;
  for (int w = w0; w < w1; ++w) {
    cum[w] = run;
    run += fmax((double)dens[w], 0.0) * sc + fl2;
  }
  if (tid == 255) cum[nw] = 1.0;
}

__global__ void mesh_place_kernel(const double *cum, int nw, double lo,
                                  double hi, int64_t M, double *E) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const double u = (j + 0.5) / (double)M;
  int a = 0, b = nw;  // largest w with cum[w] <= u
  while (b - a > 1) {
    const int mid = (a + b) >> 1;
    if (cum[mid] <= u)
      a = mid;
    else
      b = mid;
  }
  const double c0 = cum[a], c1 = cum[a + 1];
  const double f = c1 > c0 ? (u - c0) / (c1 - c0) : 0.5;
  const double h = (hi - lo) / nw;
  E[j] = lo + (a + fmin(fmax(f, 0.0), 1.0)) * h;
}

struct Mlp {
  int d_in, width, layers, prec;
  std::vector<int> din, dout;        // per layer
  std::vector<int64_t> woff, boff;   // offsets into the flat array
  int64_t n_params;
  float *p, *g, *m, *v;              // device [n_params]
  int64_t step;
  int cap_b;                         // activation capacity (batch)
  float *Z, *A, *dA, *dZ, *Y;        // device activations
  int device;
};

static unsigned g1(int64_t n) { return (unsigned)((n + 255) / 256); }

static void gemm(const Mlp &q, const float *A, int64_t sai, int64_t sak,
                 const float *B, int64_t sbk, int64_t sbj, float *C, int ldc,
                 int M, int N, int K, int acc, hipStream_t st) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  if (q.prec == 0)
    hipLaunchKernelGGL(mlp_gemm_kernel<true>, grid, dim3(256), 0, st, A, sai,
                       sak, B, sbk, sbj, C, ldc, M, N, K, acc);
  else
    hipLaunchKernelGGL(mlp_gemm_kernel<false>, grid, dim3(256), 0, st, A, sai,
                       sak, B, sbk, sbj, C, ldc, M, N, K, acc);
}

static int ensure_cap(Mlp &q, int B) {
  if (B <= q.cap_b) return RM_OK;
  for (float *x : {q.Z, q.A, q.dA, q.dZ, q.Y})
    if (x) (void)hipFree(x);
  q.Z = q.A = q.dA = q.dZ = q.Y = nullptr;
  const size_t per = (size_t)B * q.width * q.layers * sizeof(float);
  hipError_t e = hipMalloc(&q.Z, per);
  if (e == hipSuccess) e = hipMalloc(&q.A, per);
  if (e == hipSuccess) e = hipMalloc(&q.dA, (size_t)B * std::max(q.width, q.d_in) * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&q.dZ, (size_t)B * std::max(q.width, q.d_in) * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&q.Y, (size_t)B * sizeof(float));
  if (e != hipSuccess) return RM_ERR_NOMEM;
  q.cap_b = B;
  return RM_OK;
}

// Z_l / A_l of layer l live at offset l*B*width (the last layer uses width 1
// of its slot); the input is X.
static void forward(Mlp &q, const float *X, int B, hipStream_t st) {
  const float *in = X;
  int64_t ld_in = q.d_in;
  for (int l = 0; l < q.layers; ++l) {
    float *Z = q.Z + (int64_t)l * B * q.width;
    float *A = q.A + (int64_t)l * B * q.width;
    const int N = q.dout[l], K = q.din[l];
    // Z[b][j] = sum_k in[b][k] W[j][k]
    gemm(q, in, ld_in, 1, q.p + q.woff[l], 1, K, Z, N, B, N, K, 0, st);
    const int act = (l + 1 < q.layers) ? 1 : 0;
    hipLaunchKernelGGL(bias_act_kernel, dim3(g1((int64_t)B * N)), dim3(256), 0,
                       st, Z, A, q.p + q.boff[l], B, N, act);
    in = A;
    ld_in = N;
  }
}

static void backward(Mlp &q, const float *X, int B, const float *dY,
                     hipStream_t st) {
  // dZ of the last layer is dY (linear output)
  const float *dZ = dY;
  for (int l = q.layers - 1; l >= 0; --l) {
    const int N = q.dout[l], K = q.din[l];
    const float *in = (l == 0) ? X : q.A + (int64_t)(l - 1) * B * q.width;
    const int64_t ld_in = (l == 0) ? q.d_in : q.width;
    // dW[j][k] = sum_b dZ[b][j] in[b][k]
    gemm(q, dZ, 1, N, in, ld_in, 1, q.g + q.woff[l], K, N, K, B, 0, st);
    hipLaunchKernelGGL(bias_grad_kernel, dim3(g1(N)), dim3(256), 0, st, dZ,
                       q.g + q.boff[l], B, N);
    if (l == 0) break;
    // dA_{l-1}[b][k] = sum_j dZ[b][j] W[j][k]
    gemm(q, dZ, N, 1, q.p + q.woff[l], K, 1, q.dA, K, B, K, N, 0, st);
    hipLaunchKernelGGL(act_bwd_kernel, dim3(g1((int64_t)B * K)), dim3(256), 0,
                       st, q.dA, q.Z + (int64_t)(l - 1) * B * q.width, q.dZ,
                       (int64_t)B * K);
    dZ = q.dZ;
  }
}

}  // namespace rmx

using namespace rmx;

struct rm_mlp : public rmx::Mlp {};

static uint64_t splitmix(uint64_t &s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

extern "C" {

int rm_mlp_create(int32_t d_in, int32_t width, int32_t n_layers, int32_t prec,
                  uint64_t seed, rm_mlp_t *out) {
  if (!out) return (set_error(RM_ERR_ARG, "null out"), RM_ERR_ARG);
  *out = nullptr;
  if (d_in < 1 || width < 1 || n_layers < 2 || prec < 0 || prec > 1 ||
      d_in > 4096 || width > 4096 || n_layers > 16)
    return (set_error(RM_ERR_ARG, "bad MLP shape or precision"), RM_ERR_ARG);
  rm_mlp *q = new (std::nothrow) rm_mlp();
  if (!q) return (set_error(RM_ERR_NOMEM, "host allocation"), RM_ERR_NOMEM);
  q->d_in = d_in;
  q->width = width;
  q->layers = n_layers;
  q->prec = prec;
  q->step = 0;
  q->cap_b = 0;
  q->Z = q->A = q->dA = q->dZ = q->Y = nullptr;
  q->p = q->g = q->m = q->v = nullptr;
  (void)hipGetDevice(&q->device);
  int64_t off = 0;
  for (int l = 0; l < n_layers; ++l) {
    const int in = (l == 0) ? d_in : width;
    const int o = (l + 1 == n_layers) ? 1 : width;
    q->din.push_back(in);
    q->dout.push_back(o);
    q->woff.push_back(off);
    off += (int64_t)in * o;
    q->boff.push_back(off);
    off += o;
  }
  q->n_params = off;
  // He-style uniform init from a seeded splitmix64 stream
  std::vector<float> h((size_t)off, 0.0f);
  uint64_t s = seed;
  for (int l = 0; l < n_layers; ++l) {
    const double bound = std::sqrt(6.0 / q->din[l]) * (l + 1 == n_layers ? 0.1 : 1.0);
    for (int64_t i = 0; i < (int64_t)q->din[l] * q->dout[l]; ++i) {
      const double u = (splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
      h[q->woff[l] + i] = (float)((2.0 * u - 1.0) * bound);
    }
  }
  hipError_t e = hipSuccess;
  for (float **x : {&q->p, &q->g, &q->m, &q->v})
    if (e == hipSuccess) e = hipMalloc(x, (size_t)off * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(q->p, h.data(), (size_t)off * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(q->g, 0, (size_t)off * sizeof(float));
  if (e == hipSuccess) e = hipMemset(q->m, 0, (size_t)off * sizeof(float));
  if (e == hipSuccess) e = hipMemset(q->v, 0, (size_t)off * sizeof(float));
  if (e != hipSuccess) {
    for (float *x : {q->p, q->g, q->m, q->v})
      if (x) (void)hipFree(x);
    delete q;
    return (set_error(RM_ERR_NOMEM, "MLP device allocation"), RM_ERR_NOMEM);
  }
  *out = q;
  return RM_OK;
}

int rm_mlp_free(rm_mlp_t q) {
  if (!q) return RM_OK;
  (void)hipDeviceSynchronize();
  for (float *x : {q->p, q->g, q->m, q->v, q->Z, q->A, q->dA, q->dZ, q->Y})
    if (x) (void)hipFree(x);
  delete q;
  return RM_OK;
}

int rm_mlp_n_params(rm_mlp_t q, int64_t *n) {
  if (!q || !n) return (set_error(RM_ERR_ARG, "null argument"), RM_ERR_ARG);
  *n = q->n_params;
  return RM_OK;
}

int rm_mlp_get_params(rm_mlp_t q, float *dst, void *stream) {
  if (!q || !dst) return (set_error(RM_ERR_ARG, "null argument"), RM_ERR_ARG);
  hipLaunchKernelGGL(copy_f32_kernel, dim3(g1(q->n_params)), dim3(256), 0,
                     (hipStream_t)stream, q->p, dst, q->n_params);
  return hipGetLastError() == hipSuccess ? RM_OK : RM_ERR_HIP;
}

int rm_mlp_set_params(rm_mlp_t q, const float *src, void *stream) {
  if (!q || !src) return (set_error(RM_ERR_ARG, "null argument"), RM_ERR_ARG);
  hipLaunchKernelGGL(copy_f32_kernel, dim3(g1(q->n_params)), dim3(256), 0,
                     (hipStream_t)stream, src, q->p, q->n_params);
  return hipGetLastError() == hipSuccess ? RM_OK : RM_ERR_HIP;
}

int rm_mlp_forward(rm_mlp_t q, const float *X, int32_t B, float *Y,
                   void *stream) {
  if (!q || !X || !Y || B < 1)
    return (set_error(RM_ERR_ARG, "bad forward arguments"), RM_ERR_ARG);
  if (ensure_cap(*q, B)) return (set_error(RM_ERR_NOMEM, "activations"), RM_ERR_NOMEM);
  hipStream_t st = (hipStream_t)stream;
  forward(*q, X, B, st);
  const float *out = q->A + (int64_t)(q->layers - 1) * B * q->width;
  hipLaunchKernelGGL(copy_f32_kernel, dim3(g1(B)), dim3(256), 0, st, out, Y,
                     (int64_t)B);
  return hipGetLastError() == hipSuccess ? RM_OK : RM_ERR_HIP;
}

int rm_mlp_grad(rm_mlp_t q, const float *X, const float *target, int32_t B,
                float *loss, float *grad, void *stream) {
  if (!q || !X || !target || B < 1)
    return (set_error(RM_ERR_ARG, "bad grad arguments"), RM_ERR_ARG);
  if (ensure_cap(*q, B)) return (set_error(RM_ERR_NOMEM, "activations"), RM_ERR_NOMEM);
  hipStream_t st = (hipStream_t)stream;
  forward(*q, X, B, st);
  const float *out = q->A + (int64_t)(q->layers - 1) * B * q->width;
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(256), 0, st, out, target, q->Y,
                     loss, B);
  backward(*q, X, B, q->Y, st);
  if (grad)
    hipLaunchKernelGGL(copy_f32_kernel, dim3(g1(q->n_params)), dim3(256), 0,
                       st, q->g, grad, q->n_params);
  return hipGetLastError() == hipSuccess ? RM_OK : RM_ERR_HIP;
}

int rm_mlp_adam_step(rm_mlp_t q, float lr, float beta1, float beta2, float eps,
                     void *stream) {
  if (!q || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return (set_error(RM_ERR_ARG, "bad Adam arguments"), RM_ERR_ARG);
  q->step += 1;
  const float c1 = 1.f - std::pow(beta1, (float)q->step);
  const float c2 = 1.f - std::pow(beta2, (float)q->step);
  hipLaunchKernelGGL(adam_kernel, dim3(g1(q->n_params)), dim3(256), 0,
                     (hipStream_t)stream, q->p, q->g, q->m, q->v, q->n_params,
                     lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? RM_OK : RM_ERR_HIP;
}

int rm_mesh_from_density(const float *dens, int32_t nw, double lo, double hi,
                         double floor_frac, int64_t M, double *E_out,
                         void *stream) {
  if (!dens || !E_out || nw < 1 || M < 1 || !(hi > lo) ||
      !(floor_frac >= 0.0 && floor_frac <= 1.0))
    return (set_error(RM_ERR_ARG, "bad mesh arguments"), RM_ERR_ARG);
  hipStream_t st = (hipStream_t)stream;
  double *cum = nullptr;
  if (hipMallocAsync((void **)&cum, (size_t)(nw + 1) * sizeof(double), st) !=
      hipSuccess)
    return (set_error(RM_ERR_NOMEM, "cdf buffer"), RM_ERR_NOMEM);
  hipLaunchKernelGGL(density_cdf_kernel, dim3(1), dim3(256), 0, st, dens, nw,
                     floor_frac, cum);
  hipLaunchKernelGGL(mesh_place_kernel, dim3(g1(M)), dim3(256), 0, st, cum, nw,
                     lo, hi, M, E_out);
  (void)hipFreeAsync(cum, st);
  return hipGetLastError() == hipSuccess ? RM_OK : RM_ERR_HIP;
}

}  // extern "C"
