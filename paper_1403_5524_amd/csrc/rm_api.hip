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
#include <cstdlib>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <string>
#include <vector>

#include "chanfn.h"
#include "rm_internal.h"

struct rm_sym : public rmx::Sym {};

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

static int check_opts(const rm_opts *o, rm_opts *out, bool photo = false) {
  rm_opts d{};
  if (o) d = *o;
  if (d.prec < RM_PREC_FP64 || d.prec > RM_PREC_BF16X3)
    return fail(RM_ERR_ARG, "unknown precision %d", d.prec);
  if (!(d.near_delta >= 0.0) || !std::isfinite(d.near_delta))
    return fail(RM_ERR_ARG, "near_delta must be finite and >= 0");
  if (!(d.band_delta >= 0.0) || !std::isfinite(d.band_delta))
    return fail(RM_ERR_ARG, "band_delta must be finite and >= 0");
  if (d.near_delta == 0.0) d.near_delta = 1e-3;
  // the FP32-operand band: poles a few near_delta away carry the largest
  // terms of the far sum; accumulated in FP32 after them, every later term
  // is rounded against their size
  if (d.band_delta == 0.0) d.band_delta = 10.0 * d.near_delta;
  if (d.band_delta < d.near_delta)
    return fail(RM_ERR_ARG, "band_delta %g < near_delta %g", d.band_delta,
                d.near_delta);
  if (d.refine_iters < 0) return fail(RM_ERR_ARG, "refine_iters < 0");
  if (d.refine_iters == 0) d.refine_iters = 8;
  if (d.chunk < 0) return fail(RM_ERR_ARG, "chunk < 0");
  if ((d.flags & RM_FLAG_RADIATION_DAMPING) && !photo)
    return fail(RM_ERR_ARG, "RM_FLAG_RADIATION_DAMPING applies to "
                            "rm_photoionization only");
  if (d.flags & RM_FLAG_RADIATION_DAMPING) {
    if (d.prec != RM_PREC_FP64 || d.solve_fp32 ||
        (d.flags & (RM_FLAG_AUTOTUNE | RM_FLAG_PAIR_PRODUCTS)))
      return fail(RM_ERR_ARG, "the damped photoionization runs the FP64 "
                              "scaled-W pole sum and the FP64 solve only");
  }
  if (d.flags & ~(RM_FLAG_AUTOTUNE | RM_FLAG_NO_PAIR_PRODUCTS | RM_FLAG_PAIR_PRODUCTS |
                  RM_FLAG_RADIATION_DAMPING))
    return fail(RM_ERR_ARG, "unknown flags 0x%x", d.flags);
  if ((d.flags & RM_FLAG_NO_PAIR_PRODUCTS) && (d.flags & RM_FLAG_PAIR_PRODUCTS))
    return fail(RM_ERR_ARG, "RM_FLAG_NO_PAIR_PRODUCTS and RM_FLAG_PAIR_PRODUCTS together");
  if (d.solve_fp32 != 0 && d.solve_fp32 != 1)
    return fail(RM_ERR_ARG, "solve_fp32 must be 0 or 1");
  if (d.refine_iters > 100) return fail(RM_ERR_ARG, "refine_iters > 100");
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
static std::mutex g_recs_mu;  // batched inner-region solves record from threads

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
    std::lock_guard<std::mutex> lk(g_recs_mu);
    g_recs.push_back(r);
  }
  ~StageTimer() {
    if (end_) (void)hipEventRecord(end_, st_);
  }
};

ProfileScope::ProfileScope(int stage, hipStream_t st) : st_(st) {
  if (!g_prof) return;
  StageRec r{stage, nullptr, nullptr};
  if (hipEventCreate(&r.beg) != hipSuccess) return;
  if (hipEventCreate(&r.end) != hipSuccess) {
    (void)hipEventDestroy(r.beg);
    return;
  }
  (void)hipEventRecord(r.beg, st);
  end_ = r.end;
  std::lock_guard<std::mutex> lk(g_recs_mu);
  g_recs.push_back(r);
}

ProfileScope::~ProfileScope() {
  if (end_) (void)hipEventRecord(end_, st_);
}

static void clear_recs() {
  std::lock_guard<std::mutex> lk(g_recs_mu);
  for (auto &r : g_recs) {
    (void)hipEventDestroy(r.beg);
    (void)hipEventDestroy(r.end);
  }
  g_recs.clear();
}

static int free_sym(Sym *s);

// ---------------------------------------------------------------- plans
//
// A plan fixes the symmetries (ordered by cost, largest first), the chunk
// length, the workspace layout and the pole-sum work-item tables, so that
// the whole sweep is a fixed sequence of launches: per chunk one grouped
// pole-sum launch per tile variant and one persistent matching launch.

// [Aug n x 2n | K n x n | g n | v n | pivots n]: g and v serve
// photoionization, the pivots (as int) the FP32 solve's refinement
static int64_t work_doubles(int n) { return match_work_doubles(n); }
// damped photoionization: [2n x 2n real driven system, leading dimension
// 2n + 2 | R_re n x n | R_im n x n | g_re n | g_im n]
static int64_t sys_doubles_damped(int n) { return (int64_t)2 * n * (2 * n + 2); }
static int64_t work_doubles_damped(int n) {
  return sys_doubles_damped(n) + (int64_t)2 * n * n + 2 * n;
}

struct Plan {
  int device = -1;
  std::vector<const Sym *> syms;   // kernel order (cost descending)
  int n_target = 0;
  rm_opts o{};
  int64_t M = 0, C = 0;            // energies, chunk length
  int64_t work_estride = 0, chan_estride = 0;
  std::vector<int> variant;        // per symmetry (kernel order)
  // device tables
  SymDev *d_syms = nullptr;
  int64_t *d_work_off = nullptr, *d_chan_off = nullptr;
  // item tables: [variant slot][0 full chunk / 1 tail chunk]
  struct ItemSet {
    int variant;
    PsItem *d_items[2] = {nullptr, nullptr};
    int n_items[2] = {0, 0};
  };
  std::vector<ItemSet> sets;
  int64_t tail = 0;                // length of the last chunk
  int n_chunks = 0;
  // workspace
  double *work = nullptr;
  double *ext = nullptr;           // T step's complex-system pool (nullable)
  int64_t ext_estride = 0;         // doubles per slot
  int *ext_flags = nullptr;        // one per slot, 0 = free
  int ext_slots = 0;
  bool want_t = true;              // the sweep forms T (set before building)
  ChanSlot *chan = nullptr;
  int *counters = nullptr;         // one per chunk (match kernel)
  int match_grid = 0;
  bool owns_async = false;         // workspace from hipMallocAsync
  bool in_arena = false;           // tables and workspace in an Arena
  hipStream_t alloc_stream = nullptr;
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  // bound arguments
  const double *E = nullptr;
  double *omega = nullptr;
  int32_t *status = nullptr;
  // photoionization: sigma [M] (accumulated over the symmetries), e0
  double *sigma = nullptr;
  double e0 = 0.0;
  std::vector<int64_t> h_work_off;  // host copy of the workspace offsets
  bool propagate = false;           // some symmetry has outer sectors
  // damped photoionization: per-symmetry offsets of R_re and R_im
  bool damped = false;
  int64_t *d_rre_off = nullptr, *d_rim_off = nullptr;
  // rm_kmatrix-style extras (single symmetry)
  double *K_out = nullptr;
  int32_t *n_open_out = nullptr;
  double *R_out = nullptr;
  int do_t = 1;
};

static void plan_free_device(Plan &p) {
  if (p.exec) (void)hipGraphExecDestroy(p.exec);
  if (p.graph) (void)hipGraphDestroy(p.graph);
  if (p.cap_stream) (void)hipStreamDestroy(p.cap_stream);
  p.exec = nullptr;
  p.graph = nullptr;
  p.cap_stream = nullptr;
  if (p.in_arena) {  // nothing of the plan's device memory is its own
    p.sets.clear();
    p.d_syms = nullptr;
    p.d_work_off = p.d_chan_off = nullptr;
    p.work = nullptr;
    p.ext = nullptr;
    p.ext_flags = nullptr;
    p.chan = nullptr;
    p.counters = nullptr;
    return;
  }
  for (auto &set : p.sets)
    for (int t = 0; t < 2; ++t)
      if (set.d_items[t]) (void)hipFree(set.d_items[t]);
  p.sets.clear();
  void *tabs[] = {p.d_syms, p.d_work_off, p.d_chan_off, p.d_rre_off,
                  p.d_rim_off};
  for (void *q : tabs)
    if (q) (void)hipFree(q);
  p.d_syms = nullptr;
  p.d_work_off = p.d_chan_off = nullptr;
  p.d_rre_off = p.d_rim_off = nullptr;
  p.ext = nullptr;  // part of p.work
  p.ext_flags = nullptr;
  void *ws[] = {p.work, p.chan, p.counters};
  for (void *q : ws) {
    if (!q) continue;
    if (p.owns_async)
      (void)hipFreeAsync(q, p.alloc_stream);
    else
      (void)hipFree(q);
  }
  p.work = nullptr;
  p.chan = nullptr;
  p.counters = nullptr;
}

// ---- autotuner: fastest mixed tile variant per (n, N_H, precision)

struct TuneKey {
  int n, nh, prec;
  bool operator<(const TuneKey &o) const {
    return std::tie(n, nh, prec) < std::tie(o.n, o.nh, o.prec);
  }
};
static std::map<TuneKey, int> g_tuned;
static std::mutex g_tune_mu;
static bool g_tune_loaded = false;

static const char *tune_path() { return std::getenv("RM_TUNE_CACHE"); }

static void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = tune_path();
  if (!path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  int n, nh, prec, v;
  while (std::fscanf(f, "%d %d %d %d", &n, &nh, &prec, &v) == 4) {
    // an entry counts only if its variant belongs to its precision: an FP64
    // kernel launched for a mixed sweep (or the reverse) would read staged
    // operands the sweep never formed
    const bool ok64 = prec == RM_PREC_FP64 &&
                      (v == PS_F64_T32_E16 || v == PS_PD64);
    const bool okmx = (prec == RM_PREC_FP32 || prec == RM_PREC_BF16X3) &&
                      (v == PS_MX_J16_E8 || v == PS_MX_J8_E8 ||
                       v == PS_MX_J16_E4 || v == PS_PD);
    if (n > 0 && nh > 0 && (ok64 || okmx)) g_tuned[{n, nh, prec}] = v;
  }
  std::fclose(f);
}

static void tune_store() {
  const char *path = tune_path();
  if (!path) return;
  FILE *f = std::fopen(path, "w");
  if (!f) return;
  for (auto &kv : g_tuned)
    std::fprintf(f, "%d %d %d %d\n", kv.first.n, kv.first.nh, kv.first.prec,
                 kv.second);
  std::fclose(f);
}

static int default_variant(int prec) {
  return prec == RM_PREC_FP64 ? PS_F64_T32_E16 : PS_MX_J16_E8;
}

// Pair products of s for a mixed precision, formed on first use.  Returns
// true when they are (or now are) resident; false when they would not fit
// the budget (the caller then keeps the scaled-W kernels).
// Pair-product bytes held by all live symmetries of the process; the total is
// capped at 32 GB (callers hold g_tune_mu).
static double g_pd_bytes = 0.0;

static double pd_bytes(const Sym &s) {
  const double per = (s.Ph ? 4.0 : 0.0) + (s.P32 ? 4.0 : 0.0) + (s.P64 ? 8.0 : 0.0);
  return per * s.np_pad * (double)s.nh_pad;
}

static void pd_release(const Sym &s) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_pd_bytes = std::max(0.0, g_pd_bytes - pd_bytes(s));
}

static bool ensure_pd(Sym &s, int prec, hipStream_t st) {
  const bool bf = prec == RM_PREC_BF16X3, f64 = prec == RM_PREC_FP64;
  if (bf ? (s.Ph != nullptr) : f64 ? (s.P64 != nullptr) : (s.P32 != nullptr))
    return true;
  const double bytes = (f64 ? 8.0 : 4.0) * s.np_pad * (double)s.nh_pad;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return false;
  if (bytes > 8.0e9 || bytes > 0.25 * (double)free_b ||
      g_pd_bytes + bytes > 32.0e9)
    return false;
  const size_t half = (size_t)s.np_pad * s.nh_pad * sizeof(uint16_t);
  hipError_t e;
  if (bf) {
    e = hipMalloc((void **)&s.Ph, half);
    if (e == hipSuccess) e = hipMalloc((void **)&s.Pl, half);
  } else if (f64) {
    e = hipMalloc((void **)&s.P64, 4 * half);
  } else {
    e = hipMalloc((void **)&s.P32, 2 * half);
  }
  if (e == hipSuccess) e = f64 ? launch_pd64_build(s, st) : launch_pd_build(s, prec, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    if (bf) {
      if (s.Ph) (void)hipFree(s.Ph);
      if (s.Pl) (void)hipFree(s.Pl);
      s.Ph = s.Pl = nullptr;
    } else if (f64) {
      if (s.P64) (void)hipFree(s.P64);
      s.P64 = nullptr;
    } else {
      if (s.P32) (void)hipFree(s.P32);
      s.P32 = nullptr;
    }
    (void)hipGetLastError();
    return false;
  }
  g_pd_bytes += bytes;
  return true;
}

static void build_items(const Plan &p, int variant, int64_t m,
                        std::vector<PsItem> &out);

// Time every mixed variant on up to 512 energies of E (device) and keep the
// fastest.  Synchronises `st`.
static int tune_variants(const Sym &s, int prec, double delta, double band,
                         const double *E, int64_t m, hipStream_t st,
                         const std::vector<int> &cands, int *chosen);

static int tune_sym(const Sym &s, int prec, double delta, double band,
                    const double *E, int64_t m, hipStream_t st, bool with_pd,
                    int *chosen) {
  std::vector<int> c = {PS_MX_J16_E8, PS_MX_J8_E8, PS_MX_J16_E4};
  if (with_pd) c.push_back(PS_PD);
  return tune_variants(s, prec, delta, band, E, m, st, c, chosen);
}

static int tune_f64(const Sym &s, const double *E, int64_t m, hipStream_t st,
                    int *chosen) {
  return tune_variants(s, RM_PREC_FP64, 0.0, 0.0, E, m, st,
                       {PS_F64_T32_E16, PS_PD64}, chosen);
}

static int tune_variants(const Sym &s, int prec, double delta, double band,
                         const double *E, int64_t m, hipStream_t st,
                         const std::vector<int> &cands, int *chosen) {
  const int64_t mt = std::min<int64_t>(m, 512);
  const int64_t nn = (int64_t)s.n * s.n;
  double *R = nullptr;
  SymDev *dsym = nullptr;
  int64_t *doff = nullptr;
  PsItem *ditems = nullptr;
  hipEvent_t b = nullptr, e = nullptr;
  int best = cands[0];
  float best_ms = 1e30f;
  hipError_t err = hipMalloc(&R, (size_t)(mt * nn) * sizeof(double));
  if (err == hipSuccess) err = hipMalloc(&dsym, sizeof(SymDev));
  if (err == hipSuccess) err = hipMalloc(&doff, sizeof(int64_t));
  const SymDev sd = s.dev();
  const int64_t zero = 0;
  if (err == hipSuccess) err = hipMemcpy(dsym, &sd, sizeof sd, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(doff, &zero, sizeof zero, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipEventCreate(&b);
  if (err == hipSuccess) err = hipEventCreate(&e);
  for (size_t ci = 0; ci < cands.size() && err == hipSuccess; ++ci) {
    const int v = cands[ci];
    std::vector<std::pair<int, int>> tiles;
    ps_tiles(s, v, tiles);
    const int eg = ps_energy_group(v);
    std::vector<PsItem> items;
    for (auto &t : tiles)
      for (int g = 0; g < (mt + eg - 1) / eg; ++g) items.push_back({0, t.first, t.second, g});
    if (ditems) (void)hipFree(ditems);
    ditems = nullptr;
    err = hipMalloc(&ditems, items.size() * sizeof(PsItem));
    if (err == hipSuccess)
      err = hipMemcpy(ditems, items.data(), items.size() * sizeof(PsItem), hipMemcpyHostToDevice);
    PsLaunch L{};
    L.syms = dsym;
    L.items = ditems;
    L.n_items = (int)items.size();
    L.E = E;
    L.m = (int)mt;
    L.out = PsOut{R, nn, doff, 1};
    L.prec = prec;
    L.delta = delta;
    L.band = band;
    float ms_min = 1e30f;
    for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
      err = hipEventRecord(b, st);
      if (err == hipSuccess) err = launch_polesum(L, v, st);
      if (err == hipSuccess) err = hipEventRecord(e, st);
      if (err == hipSuccess) err = hipEventSynchronize(e);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, b, e);
      if (rep > 0) ms_min = std::min(ms_min, ms);  // first run warms caches
    }
    if (err == hipSuccess && ms_min < best_ms) {
      best_ms = ms_min;
      best = v;
    }
  }
  if (ditems) (void)hipFree(ditems);
  if (R) (void)hipFree(R);
  if (dsym) (void)hipFree(dsym);
  if (doff) (void)hipFree(doff);
  if (b) (void)hipEventDestroy(b);
  if (e) (void)hipEventDestroy(e);
  if (err != hipSuccess)
    return fail(RM_ERR_HIP, "autotune: %s", hipGetErrorString(err));
  *chosen = best;
  return RM_OK;
}

static int pick_variant(Sym &s, const rm_opts &o, const double *E, int64_t M,
                        hipStream_t st, int *v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  // the cache file first: tune_store rewrites it from g_tuned, so entries
  // not yet read would be lost
  tune_load();
  if (o.prec == RM_PREC_FP64) {
    // the FP64 pair-major GEMM is no faster than the scaled-W tiles on the
    // 200-channel case and costs 8 bytes per pair and pole; it is used only
    // when the autotuner times it faster
    *v = PS_F64_T32_E16;
    if (o.flags & RM_FLAG_NO_PAIR_PRODUCTS) return RM_OK;
    if (o.flags & RM_FLAG_PAIR_PRODUCTS) {
      if (ensure_pd(s, o.prec, st)) *v = PS_PD64;
      return RM_OK;
    }
    if (!(o.flags & RM_FLAG_AUTOTUNE) || M <= 0) return RM_OK;
    auto it = g_tuned.find({s.n, s.nh, o.prec});
    if (it != g_tuned.end()) {
      if (it->second == PS_F64_T32_E16 || ensure_pd(s, o.prec, st)) *v = it->second;
      return RM_OK;
    }
    if (!ensure_pd(s, o.prec, st)) return RM_OK;
    int rc = tune_f64(s, E, M, st, v);
    if (rc) return rc;
    g_tuned[{s.n, s.nh, o.prec}] = *v;
    tune_store();
    return RM_OK;
  }
  const bool pd = !(o.flags & RM_FLAG_NO_PAIR_PRODUCTS) && ensure_pd(s, o.prec, st);
  if (pd && (o.flags & RM_FLAG_PAIR_PRODUCTS)) {
    *v = PS_PD;
    return RM_OK;
  }
  auto it = g_tuned.find({s.n, s.nh, o.prec});
  if (it != g_tuned.end() && (pd || it->second != PS_PD)) {
    *v = it->second;
    return RM_OK;
  }
  if (!(o.flags & RM_FLAG_AUTOTUNE) || M <= 0) {
    *v = pd ? PS_PD : default_variant(o.prec);
    return RM_OK;
  }
  int rc = tune_sym(s, o.prec, o.near_delta, o.band_delta, E, M, st, pd, v);
  if (rc) return rc;
  if (pd) g_tuned[{s.n, s.nh, o.prec}] = *v;  // a table without the pair
  tune_store();                               // form is not cached
  return RM_OK;
}

static void build_items(const Plan &p, int variant, int64_t m,
                        std::vector<PsItem> &out) {
  out.clear();
  const int eg = ps_energy_group(variant);
  const int ngrp = (int)((m + eg - 1) / eg);
  std::vector<std::pair<int, int>> tiles;
  for (size_t q = 0; q < p.syms.size(); ++q) {
    if (p.variant[q] != variant) continue;
    ps_tiles(*p.syms[q], variant, tiles);
    for (auto &t : tiles)
      for (int g = 0; g < ngrp; ++g) out.push_back({(int)q, t.first, t.second, g});
  }
}

static int match_grid_size() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
  }
  return cus * 4;
}

// Workspace budget of a sweep: at least `base` bytes, else up to 40 % of
// the device memory free now (at most 96 GB), so that large symmetries
// still get enough energies per chunk to fill the GPU with wavefronts.
static double workspace_budget(double base) {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return base;
  return std::max(base, std::min(0.4 * (double)free_b, 96.0e9));
}

// A fixed device buffer handed out front to back (256-byte aligned pieces).
struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0;
  template <class T>
  bool take(T **out, size_t bytes) {
    const size_t at = (used + 255) & ~(size_t)255;
    if (at > cap || bytes > cap - at) return false;
    *out = (T *)(base + at);
    used = at + bytes;
    return true;
  }
};

// Variant of a symmetry for a sweep that may not allocate: the pair form
// only where its products are already resident, no autotuning.
static int pick_variant_noalloc(const Sym &s, const rm_opts &o) {
  if (o.prec == RM_PREC_FP64) {
    const bool pd = (o.flags & RM_FLAG_PAIR_PRODUCTS) && s.P64;
    return pd ? PS_PD64 : PS_F64_T32_E16;
  }
  const bool have = o.prec == RM_PREC_BF16X3 ? s.Ph != nullptr : s.P32 != nullptr;
  return (have && !(o.flags & RM_FLAG_NO_PAIR_PRODUCTS)) ? PS_PD
                                                         : default_variant(o.prec);
}

// Build a plan: orders symmetries, allocates tables and workspace.
// async: workspace from the stream-ordered allocator on st (eager calls).
// arena (non-null): every table and the workspace come from it instead, the
// tables are uploaded with copies on st, nothing is allocated, and the
// chunk length is what the arena's remaining space holds.
static int plan_build(Plan &p, const rm_sym_t *syms, int n_sym, int n_target,
                      const double *E, int64_t M, const rm_opts &o,
                      hipStream_t st, bool async, double ws_budget,
                      Arena *arena = nullptr) {
  p.o = o;
  p.n_target = n_target;
  p.M = M;
  std::vector<const Sym *> v;
  for (int q = 0; q < n_sym; ++q) v.push_back(syms[q]);
  std::stable_sort(v.begin(), v.end(), [](const Sym *x, const Sym *y) {
    const double cx = (double)x->n * x->n * x->nh + 4.0 * x->n * x->n * x->n;
    const double cy = (double)y->n * y->n * y->nh + 4.0 * y->n * y->n * y->n;
    return cx > cy;
  });
  p.syms = v;
  p.device = v[0]->device;
  p.variant.resize(v.size());
  p.damped = (o.flags & RM_FLAG_RADIATION_DAMPING) != 0;
  for (size_t q = 0; q < v.size(); ++q) {
    if (p.damped) {  // the FP64 scaled-W kernel has the damped weights
      p.variant[q] = PS_F64_T32_E16;
      continue;
    }
    if (arena) {
      p.variant[q] = pick_variant_noalloc(*v[q], o);
      continue;
    }
    int rc = pick_variant(*const_cast<Sym *>(v[q]), o, E, M, st, &p.variant[q]);
    if (rc) return rc;
  }
  std::vector<SymDev> sd;
  std::vector<int64_t> woff, coff;
  int64_t wacc = 0, cacc = 0;
  for (const Sym *s : v) {
    sd.push_back(s->dev());
    woff.push_back(wacc);
    coff.push_back(cacc);
    wacc += p.damped ? work_doubles_damped(s->n) : work_doubles(s->n);
    // the asymptotic expansion's scratch follows the symmetry's workspace
    if (!p.damped && s->n_sec > 0 && s->gl_terms > 0) {
      if (o.solve_fp32)
        return fail(RM_ERR_ARG, "the asymptotic expansion at A (rm_set_gailitis) "
                                "runs with the FP64 solve only");
      wacc += gl_doubles(s->n, s->lmax);
    }
    cacc += s->n;
  }
  p.work_estride = wacc;
  p.chan_estride = cacc;
  // the complex-system pool: slots for the largest symmetry (sweeps that
  // form T only), at most 16 GB of them
  p.ext_estride = 0;
  p.ext_slots = 0;
  if (!p.damped && p.want_t) {
    for (const Sym *s : v) p.ext_estride = std::max(p.ext_estride, t_ext_doubles(s->n));
    p.ext_slots = arena ? kTExtSlotsArena : kTExtSlots;
    while (p.ext_slots > 1 && 8.0 * p.ext_slots * (double)p.ext_estride > 16.0e9)
      p.ext_slots /= 2;
    // in an arena at most a quarter of it (none at all for very large
    // symmetries: those energies then take the route through Z)
    if (arena)
      while (p.ext_slots > 0 &&
             (8.0 * p.ext_estride + 4.0) * p.ext_slots > 0.25 * (double)arena->cap)
        p.ext_slots /= 2;
  }
  p.match_grid = match_grid_size();
  p.h_work_off = woff;
  for (const Sym *q : v) p.propagate = p.propagate || q->n_sec > 0;
  // workspace and channel slots
  const double per_energy = 8.0 * wacc + 32.0 * cacc;
  int64_t C;
  if (arena) {
    // what the arena holds after the tables (bounded by the item tables of
    // the largest chunk: at most one item per tile and energy, 16 bytes,
    // plus a counter per chunk)
    const double tables = (double)sd.size() * (sizeof(SymDev) + 16) + 65536.0;
    // less the complex-system pool and its flags
    const double room = (double)arena->cap - tables -
                        (8.0 * p.ext_estride + 4.0) * p.ext_slots - 256.0;
    double tiles = 0.0;
    {
      std::vector<std::pair<int, int>> tl;
      for (size_t q = 0; q < v.size(); ++q) {
        ps_tiles(*v[q], p.variant[q], tl);
        tiles += (double)tl.size();
      }
    }
    // per energy: workspace, slots, and the pole-sum items of a full and a
    // tail chunk (one per tile and energy group, at most one per energy),
    // plus the per-chunk counters for M / C chunks
    const double per = per_energy + 2.0 * tiles * sizeof(PsItem) + 512.0;
    C = room > per ? (int64_t)(room / per) : 0;
    if (o.chunk > 0) C = std::min<int64_t>(C, o.chunk);
    if (C < 1)
      return fail(RM_ERR_ARG, "one energy of these symmetries needs %.0f bytes "
                  "of scratch, over the %zu-byte limit", per + tables, arena->cap);
    C = std::min<int64_t>(C, 4096);
  } else {
    // up to 16384 energies per chunk (about 8 per resident wavefront of the
    // matching at 200 channels): the few energies whose T step takes the
    // complex route cost about three ordinary ones, and with only two
    // energies per wavefront a chunk would end with whichever of them came
    // last (24 % more matching time at 4096, 3 % at 16384)
    C = o.chunk > 0 ? o.chunk : (int64_t)(ws_budget / (per_energy + 64.0));
    C = std::max<int64_t>(1, std::min<int64_t>(C, p.want_t ? 16384 : 4096));
    if (o.chunk <= 0) C = std::max<int64_t>(std::min<int64_t>(64, M), C);
  }
  C = std::min<int64_t>(C, std::max<int64_t>(M, 1));
  p.C = C;
  p.n_chunks = (int)((M + C - 1) / C);
  p.tail = M - (int64_t)(p.n_chunks - 1) * C;
  p.in_arena = arena != nullptr;
  hipError_t e = hipSuccess;
  // device memory for a table: from the arena or hipMalloc
  auto get = [&](void **ptr, size_t bytes) -> hipError_t {
    if (!arena) return hipMalloc(ptr, bytes);
    return arena->take(ptr, bytes) ? hipSuccess : hipErrorOutOfMemory;
  };
  auto put = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
    return arena ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st)
                 : hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  e = get((void **)&p.d_syms, sd.size() * sizeof(SymDev));
  if (e == hipSuccess) e = get((void **)&p.d_work_off, woff.size() * sizeof(int64_t));
  if (e == hipSuccess) e = get((void **)&p.d_chan_off, coff.size() * sizeof(int64_t));
  if (e == hipSuccess) e = put(p.d_syms, sd.data(), sd.size() * sizeof(SymDev));
  if (e == hipSuccess) e = put(p.d_work_off, woff.data(), woff.size() * sizeof(int64_t));
  if (e == hipSuccess) e = put(p.d_chan_off, coff.data(), coff.size() * sizeof(int64_t));
  if (p.damped && !arena) {
    std::vector<int64_t> re(v.size()), im(v.size());
    for (size_t q = 0; q < v.size(); ++q) {
      re[q] = woff[q] + sys_doubles_damped(v[q]->n);
      im[q] = re[q] + (int64_t)v[q]->n * v[q]->n;
    }
    if (e == hipSuccess) e = get((void **)&p.d_rre_off, re.size() * sizeof(int64_t));
    if (e == hipSuccess) e = get((void **)&p.d_rim_off, im.size() * sizeof(int64_t));
    if (e == hipSuccess) e = put(p.d_rre_off, re.data(), re.size() * sizeof(int64_t));
    if (e == hipSuccess) e = put(p.d_rim_off, im.data(), im.size() * sizeof(int64_t));
  }
  std::vector<int> vars(p.variant.begin(), p.variant.end());
  std::sort(vars.begin(), vars.end());
  vars.erase(std::unique(vars.begin(), vars.end()), vars.end());
  std::vector<std::vector<PsItem>> staged;  // host tables alive until synced
  for (int var : vars) {
    if (e != hipSuccess) break;
    Plan::ItemSet set;
    set.variant = var;
    for (int t = 0; t < 2; ++t) {
      const int64_t m = (t == 0) ? C : p.tail;
      staged.emplace_back();
      std::vector<PsItem> &items = staged.back();
      build_items(p, var, m, items);
      set.n_items[t] = (int)items.size();
      if (items.empty()) continue;
      e = get((void **)&set.d_items[t], items.size() * sizeof(PsItem));
      if (e == hipSuccess)
        e = put(set.d_items[t], items.data(), items.size() * sizeof(PsItem));
      if (e != hipSuccess) break;
    }
    p.sets.push_back(set);
  }
  // the host tables go out of scope here: wait for their copies
  if (arena && e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? (arena ? RM_ERR_ARG : RM_ERR_NOMEM)
                                         : RM_ERR_HIP,
                "plan tables: %s", hipGetErrorString(e));
  const size_t wbytes = (size_t)(C * wacc) * sizeof(double);
  // the pool and its flags after the workspace, in one allocation
  const size_t xbytes = (size_t)(p.ext_slots * p.ext_estride) * sizeof(double) +
                        (size_t)p.ext_slots * sizeof(int);
  const size_t cbytes = (size_t)(C * cacc) * sizeof(ChanSlot);
  const size_t kbytes = (size_t)std::max(1, p.n_chunks) * sizeof(int);
  p.owns_async = async && !arena;
  p.alloc_stream = st;
  // the complex-system pool is carved from the end of the workspace's own
  // allocation (a part per energy there timed 4 % faster at 200 channels
  // than in an allocation of its own)
  if (arena) {
    e = arena->take(&p.work, wbytes + xbytes) && arena->take(&p.chan, cbytes) &&
                arena->take(&p.counters, kbytes)
            ? hipSuccess
            : hipErrorOutOfMemory;
    if (e != hipSuccess)
      return fail(RM_ERR_ARG, "workspace of %zu bytes does not fit the "
                  "%zu-byte scratch", wbytes + xbytes + cbytes, arena->cap);
  } else if (async) {
    e = hipMallocAsync((void **)&p.work, wbytes + xbytes, st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&p.chan, cbytes, st);
    if (e == hipSuccess) e = hipMallocAsync((void **)&p.counters, kbytes, st);
  } else {
    e = hipMalloc((void **)&p.work, wbytes + xbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&p.chan, cbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&p.counters, kbytes);
  }
  if (e == hipSuccess && p.ext_slots) {
    p.ext = p.work + C * wacc;
    p.ext_flags = (int *)(p.ext + (int64_t)p.ext_slots * p.ext_estride);
  }
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP,
                "workspace of %zu bytes: %s", wbytes + xbytes + cbytes,
                hipGetErrorString(e));
  return RM_OK;
}

// Enqueue the whole sweep of a plan on st.
static int plan_enqueue(Plan &p, hipStream_t st) {
  const int64_t P = (int64_t)p.n_target * (p.n_target + 1) / 2;
  if (p.omega) RM_HIP(launch_fill(p.omega, p.M * P, 0.0, st));
  if (p.status) RM_HIP(launch_fill_i32(p.status, p.M, 0, st));
  if (p.sigma) RM_HIP(launch_fill(p.sigma, p.M, 0.0, st));
  RM_HIP(launch_fill_i32(p.counters, std::max(1, p.n_chunks), 0, st));
  if (p.ext_flags) RM_HIP(launch_fill_i32(p.ext_flags, p.ext_slots, 0, st));
  for (int c = 0; c < p.n_chunks; ++c) {
    const int64_t c0 = (int64_t)c * p.C;
    const int64_t m = std::min(p.C, p.M - c0);
    const int t = (m == p.C) ? 0 : 1;
    {
      StageTimer tm(1, st);
      for (auto &set : p.sets) {
        PsLaunch L{};
        L.syms = p.d_syms;
        L.items = set.d_items[t];
        L.n_items = set.n_items[t];
        L.counter = nullptr;
        L.E = p.E + c0;
        L.m = (int)m;
        L.out = PsOut{p.work, p.work_estride, p.d_work_off, 2};
        L.prec = p.o.prec;
        L.delta = p.o.near_delta;
        L.band = p.o.band_delta;
        if (p.damped) {
          // real and imaginary parts of R with damped pole energies
          L.out = PsOut{p.work, p.work_estride, p.d_rre_off, 1};
          L.part = 1;
          RM_HIP(launch_polesum(L, set.variant, st));
          L.out = PsOut{p.work, p.work_estride, p.d_rim_off, 1};
          L.part = 2;
        }
        RM_HIP(launch_polesum(L, set.variant, st));
      }
      if (p.sigma && p.damped) {
        for (size_t q = 0; q < p.syms.size(); ++q) {
          const Sym &s = *p.syms[q];
          const int64_t go = p.h_work_off[q] + sys_doubles_damped(s.n) +
                             (int64_t)2 * s.n * s.n;
          RM_HIP(launch_dip_polesum(s.dev(), p.E + c0, (int)m, p.work,
                                    p.work_estride, go, st, 1));
          RM_HIP(launch_dip_polesum(s.dev(), p.E + c0, (int)m, p.work,
                                    p.work_estride, go + s.n, st, 2));
        }
      } else if (p.sigma) {
        // dipole pole sums after each symmetry's K block
        for (size_t q = 0; q < p.syms.size(); ++q) {
          const Sym &s = *p.syms[q];
          RM_HIP(launch_dip_polesum(s.dev(), p.E + c0, (int)m, p.work,
                                    p.work_estride,
                                    p.h_work_off[q] + (int64_t)3 * s.n * s.n,
                                    st));
        }
      }
    }
    if (p.R_out) {
      const Sym &s = *p.syms[0];
      RM_HIP(launch_unsort_square(s, p.work, p.work_estride, 2 * s.n,
                                  p.R_out + c0 * s.n * s.n, m, st));
    }
    MatchLaunch L{};
    L.syms = p.d_syms;
    L.n_sym = (int)p.syms.size();
    L.E = p.E + c0;
    L.m = (int)m;
    L.work = p.work;
    L.work_estride = p.work_estride;
    L.work_off = p.d_work_off;
    L.ext = p.ext;
    L.ext_estride = p.ext_estride;
    L.ext_flags = p.ext_flags;
    L.ext_slots = p.ext_slots;
    L.chan = p.chan;
    L.chan_estride = p.chan_estride;
    L.chan_off = p.d_chan_off;
    L.n_open_out = p.n_open_out ? p.n_open_out + c0 : nullptr;
    L.K_out = p.K_out ? p.K_out + c0 * p.syms[0]->n * p.syms[0]->n : nullptr;
    L.K_in = nullptr;
    L.omega = p.omega ? p.omega + c0 * P : nullptr;
    L.omega_stride = P;
    L.n_target_out = p.n_target;
    L.status = p.status ? p.status + c0 : nullptr;
    L.do_t = p.do_t;
    L.sigma = p.sigma ? p.sigma + c0 : nullptr;
    L.e0 = p.e0;
    L.counter = p.counters + c;
    L.grid = p.match_grid;
    L.solve_fp32 = p.o.solve_fp32;
    L.refine_iters = p.o.refine_iters;
    L.damped = p.damped ? 1 : 0;
    L.n_max = 0;
    for (const Sym *q : p.syms) L.n_max = std::max(L.n_max, q->n);
    if (p.propagate) {
      StageTimer tp(7, st);
      RM_HIP(launch_propagate(L, st));
    }
    StageTimer tm(2, st);
    RM_HIP(launch_match(L, st));
  }
  return RM_OK;
}

static int validate_syms(const rm_sym_t *syms, int32_t n_sym, int32_t n_target) {
  if (!syms || n_sym < 1) return fail(RM_ERR_ARG, "no symmetries");
  if (n_target < 1) return fail(RM_ERR_ARG, "n_target < 1");
  for (int q = 0; q < n_sym; ++q) {
    if (!syms[q]) return fail(RM_ERR_ARG, "null handle %d", q);
    if (syms[q]->n_target > n_target)
      return fail(RM_ERR_ARG, "symmetry %d has target level %d >= n_target %d",
                  q, syms[q]->n_target - 1, n_target);
  }
  for (int q = 0; q < n_sym; ++q) {
    int rc = check_device(syms[q]);
    if (rc) return rc;
  }
  return RM_OK;
}

static double pd_bytes(const Sym &s);
static void pd_release(const Sym &s);

static int free_sym(Sym *s) {
  if (!s) return RM_OK;
  pd_release(*s);
  void *ptrs[] = {s->E_pole, s->Wt, s->W32c, s->Whc, s->Wlc, s->e_thr,
                  s->l,      s->perm, s->inv, s->tgt,  s->ut,  s->G, s->GT,
                  s->pair_ij, s->Ph, s->Pl, s->P32, s->P64, s->dip,
                  s->prop_O, s->prop_eps, s->gam, s->gl_beta};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete[] s->h_e_thr;
  delete[] s->h_perm;
  delete s;
  return RM_OK;
}

}  // namespace rmx

using namespace rmx;

extern "C" {

const char *rm_last_error(void) { return g_err.c_str(); }

int rm_profile(int32_t enable) {
  if (enable) clear_recs();
  g_prof = enable != 0;
  return RM_OK;
}

int rm_profile_query(int32_t stage, double *total_ms, int64_t *launches) {
  if (stage < 0 || stage > 9) return fail(RM_ERR_ARG, "stage %d", stage);
  double tot = 0.0;
  int64_t cnt = 0;
  std::lock_guard<std::mutex> lk(g_recs_mu);
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
  // target level of each sorted position; the levels that hold a channel
  // and the 0/1 channel-to-level matrix over them
  std::vector<int32_t> tgt(n), ut;
  for (int i = 0; i < n; ++i) tgt[i] = d->target ? d->target[perm[i]] : perm[i];
  {
    std::vector<char> used(n_target, 0);
    for (int i = 0; i < n; ++i) used[tgt[i]] = 1;
    for (int t = 0; t < n_target; ++t)
      if (used[t]) ut.push_back(t);
  }
  const int ntu = (int)ut.size();
  std::vector<double> G, GT;
  if (ntu < n) {
    std::vector<int32_t> col_of(n_target, -1);
    for (int a = 0; a < ntu; ++a) col_of[ut[a]] = a;
    G.assign((size_t)n * ntu, 0.0);
    GT.assign((size_t)n * ntu, 0.0);
    for (int i = 0; i < n; ++i) {
      const int a = col_of[tgt[i]];
      G[(size_t)i * ntu + a] = 1.0;
      GT[(size_t)a * n + i] = 1.0;
    }
  }
  s->ntu = ntu;
  // upper-triangle channel pairs, row-major, padded to the pair block
  s->np = n * (n + 1) / 2;
  s->np_pad = (s->np + kPairBlock - 1) / kPairBlock * kPairBlock;
  std::vector<int32_t> pair_ij((size_t)s->np_pad, 0);
  {
    int q = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i; j < n; ++j) pair_ij[q++] = (i << 16) | j;
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
  RM_ALLOC_COPY(s->tgt, tgt.data(), n * sizeof(int32_t));
  RM_ALLOC_COPY(s->pair_ij, pair_ij.data(), (size_t)s->np_pad * sizeof(int32_t));
  RM_ALLOC_COPY(s->ut, ut.data(), ntu * sizeof(int32_t));
  if (ntu < n) {
    RM_ALLOC_COPY(s->G, G.data(), (size_t)n * ntu * sizeof(double));
    RM_ALLOC_COPY(s->GT, GT.data(), (size_t)n * ntu * sizeof(double));
  }
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


int rm_sweep_energies(const rm_sym_t *syms, int32_t n_sym, int32_t n_target,
                      const double *E, int64_t M, const rm_opts *opts,
                      double *omega, int32_t *status, void *stream) {
  if (M < 0) return fail(RM_ERR_ARG, "M < 0");
  rm_opts o;
  int rc = check_opts(opts, &o);
  if (rc) return rc;
  if (!syms || n_sym < 1 || n_target < 1) return validate_syms(syms, n_sym, n_target);
  for (int q = 0; q < n_sym; ++q)
    if (!syms[q]) return fail(RM_ERR_ARG, "null handle %d", q);
  if (M > 0 && (!E || !omega)) return fail(RM_ERR_ARG, "null E or omega");
  if ((rc = validate_syms(syms, n_sym, n_target))) return rc;
  if (M == 0) return RM_OK;
  hipStream_t st = (hipStream_t)stream;
  Plan p;
  rc = plan_build(p, syms, n_sym, n_target, E, M, o, st, true,
                  workspace_budget(16.0e9));
  if (!rc) {
    p.E = E;
    p.omega = omega;
    p.status = status;
    rc = plan_enqueue(p, st);
  }
  plan_free_device(p);
  return rc;
}

}  // extern "C"

namespace rmx {

// The workspace of rm_sweep_energies_noalloc: one static device array per
// GPU.  In host code `scratch` names a host-side stand-in, never the device
// memory: kernels and copies use the address hipGetSymbolAddress returns
// for the current device, looked up once per device.
static __device__ __align__(256) char scratch[RM_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, char *> g_scratch_ptr;

static int scratch_arena(Arena &a) {
  int dev = 0;
  RM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(RM_ERR_HIP, "scratch address on device %d: %s", dev,
                  hipGetErrorString(e));
    it = g_scratch_ptr.emplace(dev, (char *)ptr).first;
  }
  a.base = it->second;
  a.cap = RM_NOALLOC_SCRATCH_BYTES;
  a.used = 0;
  return RM_OK;
}

}  // namespace rmx

extern "C" {

int rm_sweep_energies_noalloc(const rm_sym_t *syms, int32_t n_sym,
                              int32_t n_target, const double *E, int64_t M,
                              const rm_opts *opts, double *omega,
                              int32_t *status, void *stream) {
  if (M < 0) return fail(RM_ERR_ARG, "M < 0");
  rm_opts o;
  int rc = check_opts(opts, &o);
  if (rc) return rc;
  if (o.flags & RM_FLAG_AUTOTUNE)
    return fail(RM_ERR_ARG, "RM_FLAG_AUTOTUNE allocates: not available "
                            "without allocation");
  if (!syms || n_sym < 1 || n_target < 1) return validate_syms(syms, n_sym, n_target);
  for (int q = 0; q < n_sym; ++q)
    if (!syms[q]) return fail(RM_ERR_ARG, "null handle %d", q);
  if (M > 0 && (!E || !omega)) return fail(RM_ERR_ARG, "null E or omega");
  if ((rc = validate_syms(syms, n_sym, n_target))) return rc;
  if (M == 0) return RM_OK;
  hipStream_t st = (hipStream_t)stream;
  Arena arena;
  if ((rc = scratch_arena(arena))) return rc;
  Plan p;
  rc = plan_build(p, syms, n_sym, n_target, E, M, o, st, false, 0.0, &arena);
  if (!rc) {
    p.E = E;
    p.omega = omega;
    p.status = status;
    rc = plan_enqueue(p, st);
  }
  plan_free_device(p);
  return rc;
}

int rm_set_propagation(rm_sym_t sym, double A, int32_t n_sec, int32_t lmax,
                       const double *beta, void *stream) {
  if (!sym) return fail(RM_ERR_ARG, "null handle");
  int rc = check_device(sym);
  if (rc) return rc;
  if (n_sec < 0 || n_sec > 100000) return fail(RM_ERR_ARG, "n_sec outside [0, 1e5]");
  if (lmax < 0 || lmax > 8) return fail(RM_ERR_ARG, "lmax outside [0, 8]");
  hipStream_t st = (hipStream_t)stream;
  RM_HIP(hipStreamSynchronize(st));  // queued sweeps may still read the old sectors
  if (n_sec == 0) {
    sym->n_sec = 0;
    sym->gl_terms = 0;
    return RM_OK;
  }
  if (!(A > sym->a) || !std::isfinite(A)) return fail(RM_ERR_ARG, "A must be finite and > a");
  const int n = sym->n;
  if (lmax > 0 && !beta) return fail(RM_ERR_ARG, "null beta");
  for (int64_t q = 0; q < (int64_t)lmax * n * n; ++q)
    if (!std::isfinite(beta[q])) return fail(RM_ERR_ARG, "beta not finite");
  for (int lam = 0; lam < lmax; ++lam)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) {
        const double x = beta[((int64_t)lam * n + i) * n + j];
        const double y = beta[((int64_t)lam * n + j) * n + i];
        if (std::fabs(x - y) > 1e-12 * std::max(1.0, std::fabs(x)))
          return fail(RM_ERR_ARG, "beta[%d] not symmetric", lam + 1);
      }
  // sorted channel order: position p holds input channel perm[p]
  std::vector<int> lsort(n);
  {
    std::vector<int32_t> lh(n);
    RM_HIP(hipMemcpy(lh.data(), sym->l, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) lsort[i] = lh[i];
  }
  const double h = (A - sym->a) / n_sec;
  const size_t nsq = (size_t)n * n;
  std::vector<double> O((size_t)(n_sec + 1) * nsq), eps((size_t)n_sec * n);
  std::vector<double> U(nsq, 0.0), Unew(nsq), Wm(nsq), T(nsq);
  for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;  // previous basis
  for (int sct = 0; sct < n_sec; ++sct) {
    const double r = sym->a + (sct + 0.5) * h;
    // W(r) in sorted order
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double w = 0.0;
        if (i == j)
          w = sym->h_e_thr[i] + lsort[i] * (lsort[i] + 1.0) / (r * r) -
              2.0 * sym->z / r;
        double rp = r * r;
        for (int lam = 0; lam < lmax; ++lam) {
          w += beta[((int64_t)lam * n + sym->h_perm[i]) * n + sym->h_perm[j]] / rp;
          rp *= r;
        }
        Wm[(size_t)i * n + j] = w;
      }
    // warm start: B = U^T W U (nearly diagonal after the first sector),
    // then cyclic Jacobi rotations B <- J^T B J, V <- V J until the
    // off-diagonal part is negligible; the sector basis is U V
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += Wm[(size_t)i * n + k] * U[(size_t)k * n + j];
        T[(size_t)i * n + j] = acc;
      }
    std::vector<double> B(nsq), V(nsq, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += U[(size_t)k * n + i] * T[(size_t)k * n + j];
        B[(size_t)i * n + j] = acc;
      }
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    double fro = 0.0;
    for (size_t q = 0; q < nsq; ++q) fro += B[q] * B[q];
    for (int sweep = 0; sweep < 60; ++sweep) {
      double off = 0.0;
      for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) off += B[(size_t)i * n + j] * B[(size_t)i * n + j];
      if (off <= 1e-32 * fro) break;
      for (int p = 0; p < n; ++p)
        for (int q = p + 1; q < n; ++q) {
          const double bpq = B[(size_t)p * n + q];
          if (bpq == 0.0) continue;
          const double bpp = B[(size_t)p * n + p], bqq = B[(size_t)q * n + q];
          // rotation zeroing (p, q): t = sgn(th) / (|th| + sqrt(th^2 + 1)),
          // th = (bqq - bpp) / (2 bpq)
          const double th = (bqq - bpp) / (2.0 * bpq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
          const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
          for (int k = 0; k < n; ++k) {  // columns p, q
            const double bkp = B[(size_t)k * n + p], bkq = B[(size_t)k * n + q];
            B[(size_t)k * n + p] = c * bkp - sn * bkq;
            B[(size_t)k * n + q] = sn * bkp + c * bkq;
          }
          for (int k = 0; k < n; ++k) {  // rows p, q
            const double bpk = B[(size_t)p * n + k], bqk = B[(size_t)q * n + k];
            B[(size_t)p * n + k] = c * bpk - sn * bqk;
            B[(size_t)q * n + k] = sn * bpk + c * bqk;
          }
          B[(size_t)p * n + q] = B[(size_t)q * n + p] = 0.0;
          for (int k = 0; k < n; ++k) {
            const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
            V[(size_t)k * n + p] = c * vkp - sn * vkq;
            V[(size_t)k * n + q] = sn * vkp + c * vkq;
          }
        }
    }
    // sector basis U_s = U V; O_s = U_prev^T U_s = V
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += U[(size_t)i * n + k] * V[(size_t)k * n + j];
        Unew[(size_t)i * n + j] = acc;
      }
    std::copy(V.begin(), V.end(), O.begin() + (size_t)sct * nsq);
    for (int i = 0; i < n; ++i) eps[(size_t)sct * n + i] = B[(size_t)i * n + i];
    U.swap(Unew);
  }
  // back to the channel basis: X <- O^T X O with O = U_last^T
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) O[(size_t)n_sec * nsq + (size_t)i * n + j] = U[(size_t)j * n + i];
  double *dO = nullptr, *de = nullptr;
  hipError_t e = hipMalloc((void **)&dO, O.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void **)&de, eps.size() * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(dO, O.data(), O.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(de, eps.data(), eps.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (dO) (void)hipFree(dO);
    if (de) (void)hipFree(de);
    return fail(e == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP,
                "propagation tables: %s", hipGetErrorString(e));
  }
  // couplings for the asymptotic expansion: row i of [n][lmax n] holds
  // beta^lam_im / A^lam (sorted order) for lam = 1..lmax
  double *dB = nullptr;
  if (lmax > 0) {
    std::vector<double> Bc((size_t)n * lmax * n);
    for (int i = 0; i < n; ++i)
      for (int lam = 0; lam < lmax; ++lam) {
        const double sc = std::pow(A, -(double)(lam + 1));
        for (int m = 0; m < n; ++m)
          Bc[((size_t)i * lmax + lam) * n + m] =
              beta[((int64_t)lam * n + sym->h_perm[i]) * n + sym->h_perm[m]] * sc;
      }
    e = hipMalloc((void **)&dB, Bc.size() * sizeof(double));
    if (e == hipSuccess)
      e = hipMemcpy(dB, Bc.data(), Bc.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      if (dB) (void)hipFree(dB);
      (void)hipFree(dO);
      (void)hipFree(de);
      return fail(e == hipErrorOutOfMemory ? RM_ERR_NOMEM : RM_ERR_HIP,
                  "propagation couplings: %s", hipGetErrorString(e));
    }
  }
  if (sym->prop_O) (void)hipFree(sym->prop_O);
  if (sym->prop_eps) (void)hipFree(sym->prop_eps);
  if (sym->gl_beta) (void)hipFree(sym->gl_beta);
  sym->prop_O = dO;
  sym->prop_eps = de;
  sym->gl_beta = dB;
  sym->lmax = lmax;
  sym->n_sec = n_sec;
  sym->A = A;
  sym->h_sec = h;
  return RM_OK;
}

int rm_set_gailitis(rm_sym_t sym, int32_t max_terms, void *stream) {
  if (!sym) return fail(RM_ERR_ARG, "null handle");
  if (max_terms < 0 || max_terms > kGlMaxTerms)
    return fail(RM_ERR_ARG, "max_terms outside [0, %d]", kGlMaxTerms);
  int rc = check_device(sym);
  if (rc) return rc;
  if (max_terms > 0 && sym->n_sec == 0)
    return fail(RM_ERR_STATE, "the asymptotic expansion needs the propagation "
                              "(rm_set_propagation) first");
  RM_HIP(hipStreamSynchronize((hipStream_t)stream));  // queued sweeps read it
  sym->gl_terms = max_terms;
  return RM_OK;
}

int rm_load_dipoles(rm_sym_t sym, const double *d, void *stream) {
  if (!sym || !d) return fail(RM_ERR_ARG, "null handle or dipoles");
  int rc = check_device(sym);
  if (rc) return rc;
  std::vector<double> h((size_t)sym->nh_pad, 0.0);
  for (int k = 0; k < sym->nh; ++k) {
    if (!std::isfinite(d[k])) return fail(RM_ERR_ARG, "dipole %d not finite", k);
    h[k] = d[k];
  }
  hipStream_t st = (hipStream_t)stream;
  // kernels already queued may still read the old vector
  RM_HIP(hipStreamSynchronize(st));
  if (!sym->dip) RM_HIP(hipMalloc((void **)&sym->dip, h.size() * sizeof(double)));
  RM_HIP(hipMemcpy(sym->dip, h.data(), h.size() * sizeof(double),
                   hipMemcpyHostToDevice));
  return RM_OK;
}

int rm_load_widths(rm_sym_t sym, const double *gamma, void *stream) {
  if (!sym || !gamma) return fail(RM_ERR_ARG, "null handle or widths");
  int rc = check_device(sym);
  if (rc) return rc;
  std::vector<double> h((size_t)sym->nh_pad, 0.0);
  for (int k = 0; k < sym->nh; ++k) {
    if (!std::isfinite(gamma[k]) || gamma[k] < 0.0)
      return fail(RM_ERR_ARG, "width %d not finite and >= 0", k);
    h[k] = gamma[k];
  }
  hipStream_t st = (hipStream_t)stream;
  RM_HIP(hipStreamSynchronize(st));  // queued kernels may read the old ones
  if (!sym->gam) RM_HIP(hipMalloc((void **)&sym->gam, h.size() * sizeof(double)));
  RM_HIP(hipMemcpy(sym->gam, h.data(), h.size() * sizeof(double),
                   hipMemcpyHostToDevice));
  return RM_OK;
}

int rm_photoionization(const rm_sym_t *syms, int32_t n_sym, const double *E,
                       int64_t M, double e0, const rm_opts *opts,
                       double *sigma, int32_t *status, void *stream) {
  if (M < 0) return fail(RM_ERR_ARG, "M < 0");
  if (!std::isfinite(e0)) return fail(RM_ERR_ARG, "e0 not finite");
  rm_opts o;
  int rc = check_opts(opts, &o, true);
  if (rc) return rc;
  if (!syms || n_sym < 1) return fail(RM_ERR_ARG, "no symmetries");
  const bool damped = (o.flags & RM_FLAG_RADIATION_DAMPING) != 0;
  int n_tgt = 1;
  for (int q = 0; q < n_sym; ++q) {
    if (!syms[q]) return fail(RM_ERR_ARG, "null handle %d", q);
    if (!syms[q]->dip)
      return fail(RM_ERR_ARG, "symmetry %d has no dipoles (rm_load_dipoles)", q);
    if (damped && !syms[q]->gam)
      return fail(RM_ERR_ARG, "symmetry %d has no radiative widths "
                  "(rm_load_widths)", q);
    if (syms[q]->n_sec > 0)
      return fail(RM_ERR_ARG, "symmetry %d has an outer-region propagation: "
                  "photoionization matches at r = a", q);
    n_tgt = std::max(n_tgt, syms[q]->n_target);
  }
  if (M > 0 && (!E || !sigma)) return fail(RM_ERR_ARG, "null E or sigma");
  if ((rc = validate_syms(syms, n_sym, n_tgt))) return rc;
  if (M == 0) return RM_OK;
  hipStream_t st = (hipStream_t)stream;
  Plan p;
  p.want_t = false;
  rc = plan_build(p, syms, n_sym, n_tgt, E, M, o, st, true,
                  workspace_budget(16.0e9));
  if (!rc) {
    p.E = E;
    p.sigma = sigma;
    p.e0 = e0;
    p.status = status;
    p.do_t = 1;
    rc = plan_enqueue(p, st);
  }
  plan_free_device(p);
  return rc;
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
  Plan p;
  p.want_t = false;
  rm_sym_t one[1] = {sym};
  rc = plan_build(p, one, 1, sym->n_target, E, m, o, st, true, 8.0e9);
  if (!rc) {
    p.E = E;
    p.status = status;
    p.K_out = K;
    p.n_open_out = n_open;
    p.R_out = R_opt;
    p.do_t = 0;
    rc = plan_enqueue(p, st);
  }
  plan_free_device(p);
  return rc;
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
  const int64_t ws = work_doubles(s.n), xs = t_ext_doubles(s.n);
  const int64_t C = std::max<int64_t>(1, std::min<int64_t>(m, (int64_t)(8.0e9 / (8.0 * ws))));
  int slots = kTExtSlots;
  while (slots > 1 && 8.0 * slots * (double)xs > 16.0e9) slots /= 2;
  DevBuf work, tabs, chan, ext;
  if ((rc = dev_alloc(work, (size_t)(C * ws) * sizeof(double), st))) return rc;
  if ((rc = dev_alloc(ext, (size_t)(slots * xs) * sizeof(double) + slots * sizeof(int), st)))
    return rc;
  int *ext_flags = (int *)((double *)ext.p + (int64_t)slots * xs);
  RM_HIP(launch_fill_i32(ext_flags, slots, 0, st));
  if ((rc = dev_alloc(chan, (size_t)(C * s.n) * sizeof(ChanSlot), st))) return rc;
  if ((rc = dev_alloc(tabs, sizeof(SymDev) + sizeof(int64_t), st))) return rc;
  const SymDev sd = s.dev();
  const int64_t zero = 0;
  RM_HIP(hipMemcpyAsync(tabs.p, &sd, sizeof sd, hipMemcpyHostToDevice, st));
  RM_HIP(hipMemcpyAsync((char *)tabs.p + sizeof(SymDev), &zero, sizeof zero,
                        hipMemcpyHostToDevice, st));
  const int64_t nn = (int64_t)s.n * s.n;
  const int64_t P = (int64_t)n_target * (n_target + 1) / 2;
  for (int64_t c0 = 0; c0 < m; c0 += C) {
    const int64_t mc = std::min(C, m - c0);
    MatchLaunch L{};
    L.syms = (const SymDev *)tabs.p;
    L.n_sym = 1;
    L.E = E + c0;
    L.m = (int)mc;
    L.work = (double *)work.p;
    L.work_estride = ws;
    L.ext = (double *)ext.p;
    L.ext_estride = xs;
    L.ext_flags = ext_flags;
    L.ext_slots = slots;
    L.n_max = s.n;
    L.work_off = (const int64_t *)((char *)tabs.p + sizeof(SymDev));
    L.chan = (ChanSlot *)chan.p;           // rank table of the K input
    L.chan_estride = s.n;
    L.chan_off = L.work_off;               // both offsets are zero
    L.K_in = K + c0 * nn;
    L.omega = omega + c0 * P;
    L.omega_stride = P;
    L.n_target_out = n_target;
    L.do_t = 1;
    RM_HIP(launch_match(L, st));
  }
  RM_HIP(hipStreamSynchronize(st));  // the host descriptor copies above
  (void)n_open;
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
  Plan p;
  p.want_t = false;
  rm_sym_t one[1] = {sym};
  rc = plan_build(p, one, 1, sym->n_target, E, m, o, st, true, 8.0e9);
  if (!rc) {
    const Sym &s = *sym;
    for (int c = 0; c < p.n_chunks && !rc; ++c) {
      const int64_t c0 = (int64_t)c * p.C;
      const int64_t mc = std::min(p.C, m - c0);
      const int t = (mc == p.C) ? 0 : 1;
      StageTimer tm(1, st);
      for (auto &set : p.sets) {
        PsLaunch L{};
        L.syms = p.d_syms;
        L.items = set.d_items[t];
        L.n_items = set.n_items[t];
        L.E = E + c0;
        L.m = (int)mc;
        L.out = PsOut{p.work, p.work_estride, p.d_work_off, 2};
        L.prec = p.o.prec;
        L.delta = p.o.near_delta;
        L.band = p.o.band_delta;
        hipError_t e = launch_polesum(L, set.variant, st);
        if (e != hipSuccess) rc = fail(RM_ERR_HIP, "pole sum: %s", hipGetErrorString(e));
      }
      if (!rc) {
        hipError_t e = launch_unsort_square(s, p.work, p.work_estride, 2 * s.n,
                                            R + c0 * s.n * s.n, mc, st);
        if (e != hipSuccess) rc = fail(RM_ERR_HIP, "unsort: %s", hipGetErrorString(e));
      }
    }
  }
  plan_free_device(p);
  return rc;
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

struct rm_plan : public rmx::Plan {};

int rm_plan_create(const rm_sym_t *syms, int32_t n_sym, int32_t n_target,
                   const double *E, int64_t M, const rm_opts *opts,
                   double *omega, int32_t *status, void *stream,
                   rm_plan_t *out) {
  if (!out) return fail(RM_ERR_ARG, "null out");
  *out = nullptr;
  if (M < 1) return fail(RM_ERR_ARG, "M < 1");
  if (!E || !omega) return fail(RM_ERR_ARG, "null E or omega");
  rm_opts o;
  int rc = check_opts(opts, &o);
  if (rc) return rc;
  if ((rc = validate_syms(syms, n_sym, n_target))) return rc;
  hipStream_t st = (hipStream_t)stream;
  rm_plan *p = new (std::nothrow) rm_plan();
  if (!p) return fail(RM_ERR_NOMEM, "host allocation");
  rc = plan_build(*p, syms, n_sym, n_target, E, M, o, st, false,
                  workspace_budget(32.0e9));
  if (!rc) {
    p->E = E;
    p->omega = omega;
    p->status = status;
    hipError_t e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      rc = fail(RM_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
    } else {
      const bool prof = g_prof;
      g_prof = false;  // no event records inside a captured graph
      rc = plan_enqueue(*p, p->cap_stream);
      g_prof = prof;
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
      p->graph = g;
      if (!rc && e2 != hipSuccess)
        rc = fail(RM_ERR_HIP, "end capture: %s", hipGetErrorString(e2));
      if (!rc) {
        e2 = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e2 != hipSuccess)
          rc = fail(RM_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e2));
      }
    }
  }
  if (rc) {
    plan_free_device(*p);
    delete p;
    return rc;
  }
  *out = p;
  return RM_OK;
}

int rm_plan_execute(rm_plan_t plan, void *stream) {
  if (!plan || !plan->exec) return fail(RM_ERR_ARG, "null plan");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RM_ERR_HIP, "hipGetDevice");
  if (dev != plan->device) return fail(RM_ERR_STATE, "plan built on device %d", plan->device);
  StageTimer tm(3, (hipStream_t)stream);
  RM_HIP(hipGraphLaunch(plan->exec, (hipStream_t)stream));
  return RM_OK;
}

int rm_plan_info(rm_plan_t plan, int64_t *chunk, int32_t *n_chunks,
                 int32_t *variants, int32_t n_variants) {
  if (!plan) return fail(RM_ERR_ARG, "null plan");
  if (chunk) *chunk = plan->C;
  if (n_chunks) *n_chunks = plan->n_chunks;
  if (variants)
    for (int q = 0; q < n_variants && q < (int)plan->variant.size(); ++q)
      variants[q] = plan->variant[q];
  return RM_OK;
}

int rm_plan_free(rm_plan_t plan) {
  if (!plan) return RM_OK;
  (void)hipDeviceSynchronize();
  plan_free_device(*plan);
  delete plan;
  return RM_OK;
}

}  // extern "C"
