// Host side of librmatrix: the C ABI declared in include/rmatrix.h.
//
// A handle keeps one symmetry on the device that loaded it, channels sorted
// by threshold (so the open channels at any energy form a prefix) and W
// staged pole-major in FP64, FP32 and split BF16.  rm_sweep_energies cuts
// the mesh into chunks that fit a workspace budget and, per chunk and per
// symmetry, enqueues channel functions -> pole sum -> matching/K/T/Omega on
// the caller's stream.  Workspace comes from the stream-ordered allocator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "chanfn.h"
#include "rm_internal.h"

namespace rmx {

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char *set_error(int code, const char *msg) {
  fail(code, "%s", msg);
  return g_err.c_str();
}

#define RM_HIP(call)                                                     \
  do {                                                                   \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess)                                                \
      return fail(e_ == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP, \
                  "%s failed: %s", #call, hipGetErrorString(e_));        \
  } while (0)

// ---------------------------------------------------------------- kernels

__global__ void chanfn_kernel(const double *E, int m, int n,
                              const double *e_thr, const int32_t *l, double z,
                              double a, ChanSlot *chan, int32_t *n_open,
                              int32_t *status) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int e = (int)(idx / n);
  const int i = (int)(idx % n);
  const double Ee = E[e];
  const double diff = Ee - e_thr[i];
  ChanSlot s;
  int bits = 0;
  if (diff > 0.0) {
    const OpenVals v = coulomb_open(l[i], z, sqrt(diff), a);
    s.d1 = v.c;
    s.d2 = a * v.cp;
    s.s = v.s;
    s.asp = a * v.sp;
    if (!v.ok) bits |= RM_E_CF_NOCONV;
  } else if (diff < 0.0) {
    const ClosedVals v = whittaker_closed(l[i], z, sqrt(-diff), a);
    s.d1 = v.e;
    s.d2 = v.ep;
    s.s = 0.0;
    s.asp = 0.0;
    if (!v.ok) bits |= RM_E_CF_NOCONV;
  } else {
    s.d1 = 1.0;
    s.d2 = 0.0;
    s.s = 0.0;
    s.asp = 0.0;
    bits |= RM_E_ON_THRESHOLD;
  }
  chan[idx] = s;
  if (i == 0) {
    int lo = 0, hi = n;  // count thresholds strictly below E
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (e_thr[mid] < Ee)
        lo = mid + 1;
      else
        hi = mid;
    }
    n_open[e] = lo;
  }
  if (bits && status) atomicOr(&status[e], bits);
}

__global__ void fill_kernel(double *p, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_i32_kernel(int32_t *p, int64_t count, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void unsort_square_kernel(const double *src, int64_t src_estride,
                                     int src_ld, double *dst, int n, int m,
                                     const int32_t *perm) {
  const int64_t total = (int64_t)m * n * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
       idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / ((int64_t)n * n);
    const int rem = (int)(idx % ((int64_t)n * n));
    const int i = rem / n, j = rem % n;
    dst[e * n * n + (int64_t)perm[i] * n + perm[j]] =
        src[e * src_estride + (int64_t)i * src_ld + j];
  }
}

__global__ void unsort_chan_kernel(const ChanSlot *chan, const int32_t *n_open,
                                   double *out, int n, int m,
                                   const int32_t *perm) {
  const int64_t total = (int64_t)m * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
       idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / n;
    const int i = (int)(idx % n);
    const ChanSlot s = chan[idx];
    double *o = out + (e * n + perm[i]) * 4;
    if (i < n_open[e]) {
      o[0] = s.s;
      o[1] = s.d1;
      o[2] = s.asp;
      o[3] = s.d2;
    } else {
      o[0] = s.d1;
      o[1] = s.d2;
      o[2] = 0.0;
      o[3] = 0.0;
    }
  }
}

static unsigned grid_for(int64_t count) {
  int64_t b = (count + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(count)), dim3(256), 0, st, p,
                     count, v);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v,
                           hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(count)), dim3(256), 0, st,
                     p, count, v);
  return hipGetLastError();
}

hipError_t launch_chanfn(const Sym &s, const double *E, int64_t m,
                         ChanSlot *chan, int32_t *n_open, int32_t *status,
                         hipStream_t st) {
  if (m <= 0) return hipSuccess;
  const int64_t total = m * s.n;
  const int64_t blocks = (total + 127) / 128;
  hipLaunchKernelGGL(chanfn_kernel, dim3((unsigned)blocks), dim3(128), 0, st,
                     E, (int)m, s.n, s.e_thr, s.l, s.z, s.a, chan, n_open,
                     status);
  return hipGetLastError();
}

hipError_t launch_unsort_square(const Sym &s, const double *src,
                                int64_t src_estride, int src_ld, double *dst,
                                int64_t m, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(unsort_square_kernel, dim3(grid_for(m * s.n * s.n)),
                     dim3(256), 0, st, src, src_estride, src_ld, dst, s.n,
                     (int)m, s.perm);
  return hipGetLastError();
}

static hipError_t launch_unsort_chan_open(const Sym &s, const ChanSlot *chan,
                                          const int32_t *n_open, int64_t m,
                                          double *out, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(unsort_chan_kernel, dim3(grid_for(m * s.n)), dim3(256), 0,
                     st, chan, n_open, out, s.n, (int)m, s.perm);
  return hipGetLastError();
}

// ---------------------------------------------------------------- helpers

static uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  const uint32_t bias = 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)((u + bias) >> 16);
}

static float bf16_to_float(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static int check_device(const Sym *s) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess)
    return fail(RM_ERR_HIP, "hipGetDevice failed");
  if (dev != s->device)
    return fail(RM_ERR_STATE, "handle loaded on device %d, current is %d",
                s->device, dev);
  return RM_OK;
}

static int check_opts(const rm_opts *o, rm_opts *out) {
  rm_opts d{};
  if (o) d = *o;
  if (d.prec < RM_PREC_FP64 || d.prec > RM_PREC_BF16X3)
    return fail(RM_ERR_ARG, "unknown precision %d", d.prec);
  if (!(d.near_delta >= 0.0) || !std::isfinite(d.near_delta))
    return fail(RM_ERR_ARG, "near_delta must be finite and >= 0");
  if (d.near_delta == 0.0) d.near_delta = 1e-3;
  if (d.refine_iters < 0) return fail(RM_ERR_ARG, "refine_iters < 0");
  if (d.refine_iters == 0) d.refine_iters = 8;
  if (d.chunk < 0) return fail(RM_ERR_ARG, "chunk < 0");
  if (d.flags != 0) return fail(RM_ERR_ARG, "flags must be 0");
  if (d.solve_fp32 != 0)
    return fail(RM_ERR_ARG, "solve_fp32 is not available: the matching "
                            "solve runs in FP64");
  *out = d;
  return RM_OK;
}

struct DevBuf {
  void *p = nullptr;
  hipStream_t st = nullptr;
  ~DevBuf() {
    if (p) (void)hipFreeAsync(p, st);
  }
};

static int dev_alloc(DevBuf &b, size_t bytes, hipStream_t st) {
  b.st = st;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMallocAsync(&b.p, bytes, st);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(e == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP,
                "workspace allocation of %zu bytes failed: %s", bytes,
                hipGetErrorString(e));
  }
  return RM_OK;
}

// ---------------------------------------------------------------- timing

struct StageRec {
  int stage;
  hipEvent_t beg, end;
};
static bool g_prof = false;
static std::vector<StageRec> g_recs;

struct StageTimer {
  hipEvent_t end_ = nullptr;
  hipStream_t st_;
  int stage_;
  StageTimer(int stage, hipStream_t st) : st_(st), stage_(stage) {
    if (!g_prof) return;
    StageRec r{stage, nullptr, nullptr};
    if (hipEventCreate(&r.beg) != hipSuccess) return;
    if (hipEventCreate(&r.end) != hipSuccess) {
      (void)hipEventDestroy(r.beg);
      return;
    }
    (void)hipEventRecord(r.beg, st);
    end_ = r.end;
    g_recs.push_back(r);
  }
  ~StageTimer() {
    if (end_) (void)hipEventRecord(end_, st_);
  }
};

static void clear_recs() {
  for (auto &r : g_recs) {
    (void)hipEventDestroy(r.beg);
    (void)hipEventDestroy(r.end);
  }
  g_recs.clear();
}

// Workspace doubles per energy: [M | B] (n x 2n) and K (n x n).
static int64_t work_doubles(int n) { return (int64_t)3 * n * n; }

static int64_t pick_chunk(int n_max, int64_t M, int32_t user_chunk) {
  if (user_chunk > 0) return std::min<int64_t>(user_chunk, M);
  const double budget = 8.0e9;  // bytes of matching workspace per chunk
  const double per = 8.0 * (double)work_doubles(n_max) + 64.0 * n_max;
  int64_t c = (int64_t)(budget / per);
  c = std::max<int64_t>(64, std::min<int64_t>(c, 4096));
  return std::min<int64_t>(c, M);
}

static int free_sym(Sym *s) {
  if (!s) return RM_OK;
  void *ptrs[] = {s->E_pole, s->Wt, s->W32c, s->Whc, s->Wlc, s->e_thr,
                  s->l,      s->perm, s->inv, s->tptr, s->tch};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete[] s->h_e_thr;
  delete[] s->h_perm;
  delete s;
  return RM_OK;
}

}  // namespace rmx

using namespace rmx;

struct rm_sym : public rmx::Sym {};

extern "C" {

const char *rm_last_error(void) { return g_err.c_str(); }

int rm_profile(int32_t enable) {
  if (enable) clear_recs();
  g_prof = enable != 0;
  return RM_OK;
}

int rm_profile_query(int32_t stage, double *total_ms, int64_t *launches) {
  if (stage < 0 || stage > 2) return fail(RM_ERR_ARG, "stage %d", stage);
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto &r : g_recs) {
    if (r.stage != stage) continue;
    float ms = 0.0f;
    RM_HIP(hipEventSynchronize(r.end));
    RM_HIP(hipEventElapsedTime(&ms, r.beg, r.end));
    tot += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return RM_OK;
}

int rm_load_poles(const rm_poles_desc *d, rm_sym_t *out, void *stream) {
  if (!d || !out) return fail(RM_ERR_ARG, "null desc or out");
  *out = nullptr;
  const int n = d->n_chan, nh = d->n_poles;
  if (n < 1 || n > 2048) return fail(RM_ERR_ARG, "n_chan=%d outside [1, 2048]", n);
  if (nh < 1) return fail(RM_ERR_ARG, "n_poles=%d < 1", nh);
  if (!d->E_pole || !d->w || !d->e_thr || !d->l)
    return fail(RM_ERR_ARG, "null input array");
  if (!(d->a > 0.0) || !std::isfinite(d->a)) return fail(RM_ERR_ARG, "a must be > 0");
  if (!(d->z >= 0.0) || !std::isfinite(d->z)) return fail(RM_ERR_ARG, "z must be >= 0");
  if (!(d->g > 0.0) || !std::isfinite(d->g)) return fail(RM_ERR_ARG, "g must be > 0");
  for (int k = 0; k < nh; ++k) {
    if (!std::isfinite(d->E_pole[k])) return fail(RM_ERR_ARG, "pole %d not finite", k);
    if (k && !(d->E_pole[k] > d->E_pole[k - 1]))
      return fail(RM_ERR_ARG, "poles not strictly ascending at %d", k);
  }
  if (std::fabs(d->E_pole[nh - 1]) >= 1e15 || std::fabs(d->E_pole[0]) >= 1e15)
    return fail(RM_ERR_ARG, "pole magnitude >= 1e15");
  const int64_t nw = (int64_t)n * nh;
  for (int64_t q = 0; q < nw; ++q)
    if (!std::isfinite(d->w[q])) return fail(RM_ERR_ARG, "amplitude %lld not finite", (long long)q);
  int n_target = 0;
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(d->e_thr[i])) return fail(RM_ERR_ARG, "threshold %d not finite", i);
    if (d->l[i] < 0 || d->l[i] > 12) return fail(RM_ERR_ARG, "l[%d]=%d outside [0,12]", i, d->l[i]);
    const int t = d->target ? d->target[i] : i;
    if (t < 0) return fail(RM_ERR_ARG, "target[%d]=%d < 0", i, t);
    n_target = std::max(n_target, t + 1);
  }
  hipStream_t st = (hipStream_t)stream;
  Sym *s = new (std::nothrow) rm_sym();
  if (!s) return fail(RM_ERR_NOMEM, "host allocation failed");
  std::memset((void *)s, 0, sizeof(Sym));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    free_sym(s);
    return fail(RM_ERR_HIP, "hipGetDevice failed");
  }
  s->device = dev;
  s->n = n;
  s->nh = nh;
  s->n_pad = (n + kChanPad - 1) / kChanPad * kChanPad;
  s->nh_pad = (nh + kPolePad - 1) / kPolePad * kPolePad;
  s->a = d->a;
  s->z = d->z;
  s->g = d->g;
  s->n_target = n_target;

  // stable sort of channels by threshold
  std::vector<int32_t> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) {
    return d->e_thr[x] < d->e_thr[y];
  });
  std::vector<int32_t> inv(n), lsrt(n);
  std::vector<double> ethr(n);
  for (int i = 0; i < n; ++i) {
    inv[perm[i]] = i;
    lsrt[i] = d->l[perm[i]];
    ethr[i] = d->e_thr[perm[i]];
  }
  // CSR of sorted positions per target level (ascending within a level)
  std::vector<int32_t> tptr(n_target + 1, 0), tch(n);
  for (int i = 0; i < n; ++i) tptr[(d->target ? d->target[perm[i]] : perm[i]) + 1]++;
  for (int t = 0; t < n_target; ++t) tptr[t + 1] += tptr[t];
  {
    std::vector<int32_t> fillp(tptr.begin(), tptr.end() - 1);
    for (int i = 0; i < n; ++i) {
      const int t = d->target ? d->target[perm[i]] : perm[i];
      tch[fillp[t]++] = i;
    }
  }
  // staged W, pole-major, zero padded
  const int64_t npad = s->n_pad, hpad = s->nh_pad;
  std::vector<double> Wt((size_t)(npad * hpad), 0.0);
  std::vector<float> W32((size_t)(npad * hpad), 0.0f);
  std::vector<uint16_t> Whi((size_t)(npad * hpad), 0), Wlo((size_t)(npad * hpad), 0);
  for (int i = 0; i < n; ++i) {
    const double *row = d->w + (int64_t)perm[i] * nh;
    for (int k = 0; k < nh; ++k) {
      const double v = row[k];
      Wt[(size_t)k * npad + i] = v;
      const size_t q = (size_t)i * hpad + k;
      W32[q] = (float)v;
      const uint16_t h = bf16_rne((float)v);
      Whi[q] = h;
      Wlo[q] = bf16_rne((float)(v - (double)bf16_to_float(h)));
    }
  }
  std::vector<double> Ep((size_t)hpad, kPadPole);
  for (int k = 0; k < nh; ++k) Ep[k] = d->E_pole[k];

  hipError_t e = hipSuccess;
#define RM_ALLOC_COPY(dst, src, bytes)                                        \
  if (e == hipSuccess) e = hipMalloc((void **)&(dst), (bytes));              \
  if (e == hipSuccess)                                                       \
    e = hipMemcpyAsync((dst), (src), (bytes), hipMemcpyHostToDevice, st);
  RM_ALLOC_COPY(s->E_pole, Ep.data(), hpad * sizeof(double));
  RM_ALLOC_COPY(s->Wt, Wt.data(), npad * hpad * sizeof(double));
  RM_ALLOC_COPY(s->W32c, W32.data(), npad * hpad * sizeof(float));
  RM_ALLOC_COPY(s->Whc, Whi.data(), npad * hpad * sizeof(uint16_t));
  RM_ALLOC_COPY(s->Wlc, Wlo.data(), npad * hpad * sizeof(uint16_t));
  RM_ALLOC_COPY(s->e_thr, ethr.data(), n * sizeof(double));
  RM_ALLOC_COPY(s->l, lsrt.data(), n * sizeof(int32_t));
  RM_ALLOC_COPY(s->perm, perm.data(), n * sizeof(int32_t));
  RM_ALLOC_COPY(s->inv, inv.data(), n * sizeof(int32_t));
  RM_ALLOC_COPY(s->tptr, tptr.data(), (n_target + 1) * sizeof(int32_t));
  RM_ALLOC_COPY(s->tch, tch.data(), n * sizeof(int32_t));
#undef RM_ALLOC_COPY
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    free_sym(s);
    return fail(e == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP,
                "rm_load_poles: %s", hipGetErrorString(e));
  }
  s->h_e_thr = new double[n];
  s->h_perm = new int32_t[n];
  std::memcpy(s->h_e_thr, ethr.data(), n * sizeof(double));
  std::memcpy(s->h_perm, perm.data(), n * sizeof(int32_t));
  *out = static_cast<rm_sym *>(s);
  return RM_OK;
}

int rm_free(rm_sym_t sym) {
  if (!sym) return RM_OK;
  (void)hipDeviceSynchronize();
  return free_sym(sym);
}

int rm_sym_info(rm_sym_t sym, int32_t *n_chan, int32_t *n_poles,
                int32_t *n_target) {
  if (!sym) return fail(RM_ERR_ARG, "null handle");
  if (n_chan) *n_chan = sym->n;
  if (n_poles) *n_poles = sym->nh;
  if (n_target) *n_target = sym->n_target;
  return RM_OK;
}

static int polesum_dispatch(const Sym &s, const rm_opts &o, const double *E,
                            int64_t m, double *R, int64_t estride, int ld,
                            hipStream_t st) {
  hipError_t e;
  if (o.prec == RM_PREC_FP64)
    e = launch_polesum_f64(s, E, m, R, estride, ld, st);
  else
    e = launch_polesum_mixed(s, o.prec, o.near_delta, E, m, R, estride, ld, st);
  if (e != hipSuccess)
    return fail(RM_ERR_HIP, "pole-sum launch failed: %s", hipGetErrorString(e));
  return RM_OK;
}

int rm_sweep_energies(const rm_sym_t *syms, int32_t n_sym, int32_t n_target,
                      const double *E, int64_t M, const rm_opts *opts,
                      double *omega, int32_t *status, void *stream) {
  if (!syms || n_sym < 1) return fail(RM_ERR_ARG, "no symmetries");
  if (n_target < 1) return fail(RM_ERR_ARG, "n_target < 1");
  if (M < 0) return fail(RM_ERR_ARG, "M < 0");
  if (M > 0 && (!E || !omega)) return fail(RM_ERR_ARG, "null E or omega");
  rm_opts o;
  int rc = check_opts(opts, &o);
  if (rc) return rc;
  int n_max = 0;
  for (int q = 0; q < n_sym; ++q) {
    if (!syms[q]) return fail(RM_ERR_ARG, "null handle %d", q);
    if ((rc = check_device(syms[q]))) return rc;
    if (syms[q]->n_target > n_target)
      return fail(RM_ERR_ARG, "symmetry %d has target level %d >= n_target %d",
                  q, syms[q]->n_target - 1, n_target);
    n_max = std::max(n_max, syms[q]->n);
  }
  if (M == 0) return RM_OK;
  hipStream_t st = (hipStream_t)stream;
  const int64_t P = (int64_t)n_target * (n_target + 1) / 2;
  RM_HIP(launch_fill(omega, M * P, 0.0, st));
  if (status) RM_HIP(launch_fill_i32(status, M, 0, st));
  const int64_t C = pick_chunk(n_max, M, o.chunk);
  const int64_t wstride = work_doubles(n_max);
  DevBuf work, chan, nopen;
  if ((rc = dev_alloc(work, (size_t)(C * wstride) * sizeof(double), st))) return rc;
  if ((rc = dev_alloc(chan, (size_t)(C * n_max) * sizeof(ChanSlot), st))) return rc;
  if ((rc = dev_alloc(nopen, (size_t)C * sizeof(int32_t), st))) return rc;
  for (int64_t c0 = 0; c0 < M; c0 += C) {
    const int64_t m = std::min(C, M - c0);
    for (int q = 0; q < n_sym; ++q) {
      const Sym &s = *syms[q];
      const int64_t ws = work_doubles(s.n);
      {
        StageTimer t(0, st);
        RM_HIP(launch_chanfn(s, E + c0, m, (ChanSlot *)chan.p,
                             (int32_t *)nopen.p, status ? status + c0 : nullptr,
                             st));
      }
      {
        StageTimer t(1, st);
        if ((rc = polesum_dispatch(s, o, E + c0, m, (double *)work.p, ws,
                                   2 * s.n, st)))
          return rc;
      }
      MatchArgs a{};
      a.chan = (const ChanSlot *)chan.p;
      a.n_open = (const int32_t *)nopen.p;
      a.work = (double *)work.p;
      a.work_stride = ws;
      a.m = (int)m;
      a.K_out = nullptr;
      a.omega = omega + c0 * P;
      a.omega_stride = P;
      a.n_target_out = n_target;
      a.status = status ? status + c0 : nullptr;
      a.do_t = 1;
      a.solve_fp32 = o.solve_fp32;
      a.refine_iters = o.refine_iters;
      StageTimer t(2, st);
      RM_HIP(launch_match(s, a, st));
    }
  }
  return RM_OK;
}

int rm_kmatrix(rm_sym_t sym, const double *E, int64_t m, const rm_opts *opts,
               double *K, int32_t *n_open, double *R_opt, int32_t *status,
               void *stream) {
  if (!sym) return fail(RM_ERR_ARG, "null handle");
  if (m < 0) return fail(RM_ERR_ARG, "m < 0");
  if (m > 0 && (!E || !K || !n_open)) return fail(RM_ERR_ARG, "null E, K or n_open");
  rm_opts o;
  int rc = check_opts(opts, &o);
  if (rc) return rc;
  if ((rc = check_device(sym))) return rc;
  if (m == 0) return RM_OK;
  hipStream_t st = (hipStream_t)stream;
  const Sym &s = *sym;
  if (status) RM_HIP(launch_fill_i32(status, m, 0, st));
  const int64_t C = pick_chunk(s.n, m, o.chunk);
  const int64_t ws = work_doubles(s.n);
  DevBuf work, chan;
  if ((rc = dev_alloc(work, (size_t)(C * ws) * sizeof(double), st))) return rc;
  if ((rc = dev_alloc(chan, (size_t)(C * s.n) * sizeof(ChanSlot), st))) return rc;
  const int64_t nn = (int64_t)s.n * s.n;
  for (int64_t c0 = 0; c0 < m; c0 += C) {
    const int64_t mc = std::min(C, m - c0);
    RM_HIP(launch_chanfn(s, E + c0, mc, (ChanSlot *)chan.p, n_open + c0,
                         status ? status + c0 : nullptr, st));
    if ((rc = polesum_dispatch(s, o, E + c0, mc, (double *)work.p, ws, 2 * s.n, st)))
      return rc;
    if (R_opt)
      RM_HIP(launch_unsort_square(s, (const double *)work.p, ws, 2 * s.n,
                                  R_opt + c0 * nn, mc, st));
    MatchArgs a{};
    a.chan = (const ChanSlot *)chan.p;
    a.n_open = n_open + c0;
    a.work = (double *)work.p;
    a.work_stride = ws;
    a.m = (int)mc;
    a.K_out = K + c0 * nn;
    a.omega = nullptr;
    a.n_target_out = s.n_target;
    a.status = status ? status + c0 : nullptr;
    a.do_t = 0;
    a.solve_fp32 = o.solve_fp32;
    a.refine_iters = o.refine_iters;
    RM_HIP(launch_match(s, a, st));
  }
  return RM_OK;
}

int rm_collision_strengths(rm_sym_t sym, const double *K, const int32_t *n_open,
                           const double *E, int64_t m, int32_t n_target,
                           double *omega, void *stream) {
  if (!sym) return fail(RM_ERR_ARG, "null handle");
  if (m < 0) return fail(RM_ERR_ARG, "m < 0");
  if (n_target < sym->n_target)
    return fail(RM_ERR_ARG, "n_target %d below the handle's %d levels", n_target,
                sym->n_target);
  if (m > 0 && (!K || !n_open || !E || !omega)) return fail(RM_ERR_ARG, "null pointer");
  int rc = check_device(sym);
  if (rc) return rc;
  if (m == 0) return RM_OK;
  hipStream_t st = (hipStream_t)stream;
  const Sym &s = *sym;
  const int64_t C = pick_chunk(s.n, m, 0);
  const int64_t ws = work_doubles(s.n);
  DevBuf work;
  if ((rc = dev_alloc(work, (size_t)(C * ws) * sizeof(double), st))) return rc;
  const int64_t nn = (int64_t)s.n * s.n;
  const int64_t P = (int64_t)n_target * (n_target + 1) / 2;
  for (int64_t c0 = 0; c0 < m; c0 += C) {
    const int64_t mc = std::min(C, m - c0);
    RM_HIP(launch_t_omega_from_k(s, K + c0 * nn, n_open + c0, mc, (double *)work.p,
                                 ws, omega + c0 * P, n_target, st));
  }
  return RM_OK;
}

int rm_rmatrix(rm_sym_t sym, const double *E, int64_t m, const rm_opts *opts,
               double *R, void *stream) {
  if (!sym) return fail(RM_ERR_ARG, "null handle");
  if (m < 0) return fail(RM_ERR_ARG, "m < 0");
  if (m > 0 && (!E || !R)) return fail(RM_ERR_ARG, "null E or R");
  rm_opts o;
  int rc = check_opts(opts, &o);
  if (rc) return rc;
  if ((rc = check_device(sym))) return rc;
  if (m == 0) return RM_OK;
  hipStream_t st = (hipStream_t)stream;
  const Sym &s = *sym;
  const int64_t nn = (int64_t)s.n * s.n;
  const int64_t C = std::min<int64_t>(m, std::max<int64_t>(16, (int64_t)(4.0e9 / (8.0 * nn))));
  DevBuf work;
  if ((rc = dev_alloc(work, (size_t)(C * nn) * sizeof(double), st))) return rc;
  for (int64_t c0 = 0; c0 < m; c0 += C) {
    const int64_t mc = std::min(C, m - c0);
    if ((rc = polesum_dispatch(s, o, E + c0, mc, (double *)work.p, nn, s.n, st)))
      return rc;
    RM_HIP(launch_unsort_square(s, (const double *)work.p, nn, s.n, R + c0 * nn,
                                mc, st));
  }
  return RM_OK;
}

int rm_channel_functions(rm_sym_t sym, const double *E, int64_t m, double *out,
                         int32_t *status, void *stream) {
  if (!sym) return fail(RM_ERR_ARG, "null handle");
  if (m < 0) return fail(RM_ERR_ARG, "m < 0");
  if (m > 0 && (!E || !out)) return fail(RM_ERR_ARG, "null E or out");
  int rc = check_device(sym);
  if (rc) return rc;
  if (m == 0) return RM_OK;
  hipStream_t st = (hipStream_t)stream;
  const Sym &s = *sym;
  if (status) RM_HIP(launch_fill_i32(status, m, 0, st));
  DevBuf chan, nopen;
  if ((rc = dev_alloc(chan, (size_t)(m * s.n) * sizeof(ChanSlot), st))) return rc;
  if ((rc = dev_alloc(nopen, (size_t)m * sizeof(int32_t), st))) return rc;
  RM_HIP(launch_chanfn(s, E, m, (ChanSlot *)chan.p, (int32_t *)nopen.p, status, st));
  RM_HIP(launch_unsort_chan_open(s, (const ChanSlot *)chan.p,
                                 (const int32_t *)nopen.p, m, out, st));
  return RM_OK;
}

}  // extern "C"
