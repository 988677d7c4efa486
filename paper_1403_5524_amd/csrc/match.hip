// Matching, K-matrix, T-matrix and collision strengths: one wavefront per
// energy.
//
// With channels sorted by threshold the open channels at energy E are the
// prefix P = [0, n_o).  For each open channel j the solution has open parts
// s_i d_ij + c_i K_ij and closed parts e_i X_ij; the R-matrix relation
// u(a) = R a u'(a) becomes the linear system
//     (D1 - R D2) [K; X] = R[:, P] diag(a s'_P) - [diag(s_P); 0]
// with D1 = diag(c_P, e_Q), D2 = diag(a c'_P, a e'_Q) -- no division by any
// channel function.  Then, with K symmetrised,
//     (1 + K^2) Y = K,  Q = K Y,  T = 2(X - 1) + 2iY, X = (1 + K^2)^-1
// so |T_ij|^2 = 4 (Y_ij^2 + Q_ij^2), and
//     Omega(t, u) += (g/2) sum_{i in t, j in u, open} |T_ij|^2.
//
// Each wavefront owns one energy at a time and loops over every symmetry;
// it owns that energy's Omega row, so symmetries add without atomics and in
// a fixed order.  The dense algebra is wavefront-local, in a per-energy
// global workspace (row-major, leading dimension 2n): blocked right-looking
// LU with partial pivoting (panels of 16 columns), trailing updates and
// products as 16 x 16 FP64 MFMA blocks (v_mfma_f64_16x16x4f64).
//
// The workspace of one energy is far larger than a CU's caches, so this
// code is bound by memory latency, not arithmetic.  Every pass is therefore
// written as "issue all loads of a batch, then compute, then store": the
// compiler cannot move a load above a store it cannot prove disjoint, so a
// read-modify-write loop written element by element would pay one full
// round trip per element.  GEMM tiles load A, B and C together and
// prefetch the next tile before storing the current one.
//
// Lanes of a wavefront run in lockstep, so ordering between lanes needs only
// a memory fence and a scheduling barrier -- no workgroup barrier anywhere.
// Wavefronts pull energies from an atomic counter (persistent grid).
#include <algorithm>

#include "chanfn.h"
#include "rm_internal.h"

namespace rmx {

constexpr int WT = 64;   // lanes per wavefront
constexpr int NB = 16;   // panel (factorisation) width
constexpr int NB2 = 32;  // update width: two panels per trailing update
constexpr int WPB = kMatchWpb;   // wavefronts per workgroup
constexpr int UNR = 4;   // independent elements per lane per batch

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Element types of the wavefront linear algebra: FP64 (the default path) and
// FP32 (the factorisation of the FP32 solve, refined in FP64).  The 16x16x4
// MFMAs of both read A[i][k] and B[k][j] at i = j = lane % 16, k = lane / 16;
// their 16x16 results differ in layout: FP64 row kq + 4r, FP32 row 4kq + r
// of register r (kq = lane / 16).
template <class T>
struct Mx;
template <>
struct Mx<double> {
  typedef d4 acc;
  __device__ static inline acc mfma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int kq, int r) { return kq + 4 * r; }
};
template <>
struct Mx<float> {
  typedef f4 acc;
  __device__ static inline acc mfma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int kq, int r) { return 4 * kq + r; }
};

// Per-wavefront LDS: the diagonal block of the current two panels, its
// inverse, and the row moves of their interchanges.
struct WaveLds {
  double T[NB2][NB2 + 1];
  double Ti[NB2][NB2 + 1];  // its inverse
  int piv[NB2];   // pivot row chosen at each column of the block
  int srcp[NB2];  // after the interchanges, block row q holds old row srcp[q]
  int opos[NB2];  // rows below the block that receive another row ...
  int osrc[NB2];  // ... namely old row osrc[m]
  int nout;
};

__device__ inline int lane_id() { return threadIdx.x & (WT - 1); }

// Make this lane's earlier global writes visible to the other lanes of the
// wavefront and keep the compiler from moving memory operations across.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ inline double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Wavefront argmax of a = |v| (ties -> smaller index), carrying v.
template <class T>
__device__ inline void wave_argmax(T &a, T &v, int &idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const T oa = __shfl_xor(a, off);
    const T ov = __shfl_xor(v, off);
    const int oi = __shfl_xor(idx, off);
    if (oa > a || (oa == a && oi < idx)) {
      a = oa;
      v = ov;
      idx = oi;
    }
  }
}

__device__ inline int wave_or(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off);
  return v;
}

// ---------------------------------------------------------------------------
// GEMM, wavefront-local, operands in global memory.
//   MODE 0: C -= A B  (the rank-16 and rank-32 updates of the LU)
//   MODE 1: C = A B + I
//   MODE 2: C = A B
// The wavefront walks 32 x 32 output tiles (2 x 2 MFMA blocks sharing their
// A and B fragments) in k-steps of 16.
template <class T>
struct Frag {
  T a[4][2], b[4][2];
};

// Operand storage flags of wave_gemm.
constexpr int G_TA = 1;     // A[i][k] stored at A[k * lda + i]
constexpr int G_TB = 2;     // B[k][j] stored at B[j * ldb + k]
constexpr int G_LOWER = 4;  // only the tiles of C that meet its lower triangle
constexpr int G_BSYM = 8;   // B symmetric, only its lower triangle stored
constexpr int G_KTRI = 16;  // A^T with A lower triangular (wave_gemm_wide,
                            // with G_TA): a tile's sum starts at its first row

template <int FL, class T>
__device__ inline void frag_load(Frag<T> &f, const T *A, int lda,
                                 const T *B, int ldb, int rows, int cols,
                                 int kd, int rb, int cb, int k0) {
  const int lane = lane_id();
  const int col = lane & 15, kq = lane >> 4;
  const int ra0 = rb + col, ra1 = ra0 + 16, c0 = cb + col, c1 = c0 + 16;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = k0 + 4 * s + kq;
    const bool kv = k < kd;
    if (FL & G_TA) {
      f.a[s][0] = (kv && ra0 < rows) ? A[(int64_t)k * lda + ra0] : T(0);
      f.a[s][1] = (kv && ra1 < rows) ? A[(int64_t)k * lda + ra1] : T(0);
    } else {
      f.a[s][0] = (kv && ra0 < rows) ? A[(int64_t)ra0 * lda + k] : T(0);
      f.a[s][1] = (kv && ra1 < rows) ? A[(int64_t)ra1 * lda + k] : T(0);
    }
    if (FL & G_TB) {
      f.b[s][0] = (kv && c0 < cols) ? B[(int64_t)c0 * ldb + k] : T(0);
      f.b[s][1] = (kv && c1 < cols) ? B[(int64_t)c1 * ldb + k] : T(0);
    } else {
      f.b[s][0] = (kv && c0 < cols) ? B[(int64_t)k * ldb + c0] : T(0);
      f.b[s][1] = (kv && c1 < cols) ? B[(int64_t)k * ldb + c1] : T(0);
    }
  }
}

// C tile in the result layout of the type's 16x16x4 MFMA (Mx<T>::row).
template <class T>
__device__ inline void ctile_load(T (&c)[2][2][4], const T *C,
                                  int ldc, int rows, int cols, int rb, int cb) {
  const int lane = lane_id();
  const int col = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = rb + 16 * x + Mx<T>::row(kq, r), j = cb + 16 * y + col;
        c[x][y][r] = (i < rows && j < cols) ? C[(int64_t)i * ldc + j] : T(0);
      }
}

// Next tile index after t (row-major over 32 x 32 tiles), skipping the
// tiles strictly above the diagonal when only the lower triangle is wanted.
template <int FL>
__device__ inline int gemm_next_tile(int t, int nct, int ntile) {
  ++t;
  if (FL & G_LOWER)
    while (t < ntile && (t % nct) > (t / nct)) ++t;
  return t;
}

template <int MODE, int FL = 0, class T = double>
__device__ void wave_gemm(T *C, int ldc, const T *A, int lda,
                          const T *B, int ldb, int rows, int cols,
                          int kd) {
  typedef typename Mx<T>::acc acc_t;
  const int lane = lane_id();
  const int col = lane & 15, kq = lane >> 4;
  const int nct = (cols + 31) >> 5;
  const int ntile = ((rows + 31) >> 5) * nct;
  const int nk = max(1, (kd + 15) >> 4);
  if (ntile > 0) {
    Frag<T> cur, nxt;
    T cv[2][2][4], cn[2][2][4];
    frag_load<FL>(cur, A, lda, B, ldb, rows, cols, kd, 0, 0, 0);
    if (MODE == 0) ctile_load(cv, C, ldc, rows, cols, 0, 0);
    for (int t = 0; t < ntile;) {
      const int tn = gemm_next_tile<FL>(t, nct, ntile);
      const int rb = (t / nct) * 32, cb = (t % nct) * 32;
      acc_t acc[2][2];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = acc_t{0, 0, 0, 0};
      for (int kc = 0; kc < nk; ++kc) {
        // prefetch: the next k-step of this tile, else the next tile (whose
        // A, B and C do not overlap this tile's C)
        if (kc + 1 < nk) {
          frag_load<FL>(nxt, A, lda, B, ldb, rows, cols, kd, rb, cb, (kc + 1) * 16);
        } else if (tn < ntile) {
          const int rn = (tn / nct) * 32, cnb = (tn % nct) * 32;
          frag_load<FL>(nxt, A, lda, B, ldb, rows, cols, kd, rn, cnb, 0);
          if (MODE == 0) ctile_load(cn, C, ldc, rows, cols, rn, cnb);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
              acc[x][y] = Mx<T>::mfma(cur.a[s][x], cur.b[s][y], acc[x][y]);
        cur = nxt;
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = rb + 16 * x + Mx<T>::row(kq, r), j = cb + 16 * y + col;
            if (i >= rows || j >= cols) continue;
            T v = acc[x][y][r];
            if (MODE == 0) v = cv[x][y][r] - v;
            if (MODE == 1 && i == j) v += T(1);
            C[(int64_t)i * ldc + j] = v;
          }
      if (MODE == 0) {
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) cv[x][y][r] = cn[x][y][r];
      }
      t = tn;
    }
  }
  wave_sync();
}

// Wide form: output tiles of (16 BM) x (16 BN), so each A row panel is read
// once per 16 BN columns and each B column panel once per 16 BM rows (the
// 32 x 32 tiles above read both twice as often).  MODE 0 loads C into the
// accumulators and subtracts A B through them (no separate C registers;
// the next tile's C is prefetched), MODE 1 starts from the identity, MODE 2
// from zero.  With G_LOWER only tiles whose first column is on or left of
// their last row are formed.  G_BSYM reads B[k][j] from B's lower triangle;
// G_KTRI skips the k-steps below the tile's first row (they multiply the
// zeros above the diagonal of a lower-triangular A stored transposed).
template <int MODE, int FL, int BM, int BN, class T = double>
__device__ void wave_gemm_wide(T *C, int ldc, const T *A, int lda,
                               const T *B, int ldb, int rows, int cols,
                               int kd) {
  typedef typename Mx<T>::acc acc_t;
  constexpr int TH = 16 * BM, TW = 16 * BN;
  const int lane = lane_id();
  const int col = lane & 15, kq = lane >> 4;
  const int nct = (cols + TW - 1) / TW;
  const int ntile = ((rows + TH - 1) / TH) * nct;
  const int nk = max(1, (kd + 15) >> 4);
  auto skip = [&](int t) {
    return (FL & G_LOWER) && (t % nct) * TW > (t / nct) * TH + TH - 1;
  };
  auto next = [&](int t) {
    ++t;
    while (t < ntile && skip(t)) ++t;
    return t;
  };
  // first k-step of tile t
  auto kfirst = [&](int t) {
    return (FL & G_KTRI) ? min((t / nct) * TH, kd) >> 4 : 0;
  };
  // fragments of k-step k0 for the tile at (rb, cb)
  auto fload = [&](T (&a)[4][BM], T (&b)[4][BN], int rb, int cb, int k0) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int k = k0 + 4 * s4 + kq;
      const bool kv = k < kd;
#pragma unroll
      for (int x = 0; x < BM; ++x) {
        const int i = rb + 16 * x + col;
        a[s4][x] = (kv && i < rows)
                       ? ((FL & G_TA) ? A[(int64_t)k * lda + i] : A[(int64_t)i * lda + k])
                       : T(0);
      }
#pragma unroll
      for (int y = 0; y < BN; ++y) {
        const int j = cb + 16 * y + col;
        const bool up = (FL & G_TB) || ((FL & G_BSYM) && k < j);
        b[s4][y] = (kv && j < cols)
                       ? (up ? B[(int64_t)j * ldb + k] : B[(int64_t)k * ldb + j])
                       : T(0);
      }
    }
  };
  auto cload = [&](T (&c)[BM][BN][4], int rb, int cb) {
#pragma unroll
    for (int x = 0; x < BM; ++x)
#pragma unroll
      for (int y = 0; y < BN; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rb + 16 * x + Mx<T>::row(kq, r), j = cb + 16 * y + col;
          c[x][y][r] = (i < rows && j < cols) ? C[(int64_t)i * ldc + j] : T(0);
        }
  };
  int t = skip(0) ? next(0) : 0;
  if (t < ntile) {
    T ca[4][BM], cbf[4][BN], na[4][BM], nb[4][BN];
    T cc[BM][BN][4];
    fload(ca, cbf, (t / nct) * TH, (t % nct) * TW, 16 * kfirst(t));
    while (t < ntile) {
      const int tn = next(t);
      const int rb = (t / nct) * TH, cb = (t % nct) * TW;
      if (MODE == 0) cload(cc, rb, cb);
      acc_t acc[BM][BN];
#pragma unroll
      for (int x = 0; x < BM; ++x)
#pragma unroll
        for (int y = 0; y < BN; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            T v = T(0);
            if (MODE == 0) v = cc[x][y][r];
            if (MODE == 1)
              v = (rb + 16 * x + Mx<T>::row(kq, r) == cb + 16 * y + col) ? T(1) : T(0);
            acc[x][y][r] = v;
          }
      for (int kc = kfirst(t); kc < nk; ++kc) {
        if (kc + 1 < nk) {
          fload(na, nb, rb, cb, (kc + 1) * 16);
        } else if (tn < ntile) {
          fload(na, nb, (tn / nct) * TH, (tn % nct) * TW, 16 * kfirst(tn));
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
          for (int x = 0; x < BM; ++x)
#pragma unroll
            for (int y = 0; y < BN; ++y)
              acc[x][y] = Mx<T>::mfma(MODE == 0 ? -ca[s4][x] : ca[s4][x],
                                      cbf[s4][y], acc[x][y]);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
#pragma unroll
          for (int x = 0; x < BM; ++x) ca[s4][x] = na[s4][x];
#pragma unroll
          for (int y = 0; y < BN; ++y) cbf[s4][y] = nb[s4][y];
        }
      }
#pragma unroll
      for (int x = 0; x < BM; ++x)
#pragma unroll
        for (int y = 0; y < BN; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = rb + 16 * x + Mx<T>::row(kq, r), j = cb + 16 * y + col;
            if (i < rows && j < cols) C[(int64_t)i * ldc + j] = acc[x][y][r];
          }
      t = tn;
    }
  }
  wave_sync();
}

// ---------------------------------------------------------------------------
// LU with partial pivoting.

// Factor columns [j0, j0 + jb) (jb <= 16) of rows [j0, na) in place;
// interchanges swap the row segments [sw0, j0 + jb) (the panel and the L
// columns of an earlier panel of the same block); pivots -> W.piv[po + .].
// Returns 1 if a pivot was zero or not a number.
template <class T>
__device__ int wave_panel(T *A, int na, int ld, int j0, int jb, int sw0,
                          int po, WaveLds &W) {
  const int lane = lane_id();
  int flag = 0;
#pragma unroll 1
  for (int jj = 0; jj < jb; ++jj) {
    const int col = j0 + jj;
    T ba = T(-1), bv = T(0);
    int bi = na;
    for (int r0 = col + lane; r0 < na; r0 += UNR * WT) {
      T v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int r = r0 + u * WT;
        v[u] = r < na ? A[(int64_t)r * ld + col] : T(0);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int r = r0 + u * WT;
        if (r < na && fabs(v[u]) > ba) {
          ba = fabs(v[u]);
          bv = v[u];
          bi = r;
        }
      }
    }
    wave_argmax(ba, bv, bi);
    int pr = bi;
    T pv = bv;
    if (pr >= na) {  // every candidate is NaN
      pr = col;
      pv = (T)__builtin_nan("");
    }
    if (lane == 0) W.piv[po + jj] = pr;
    // swap the segments [sw0, j0 + jb) of rows col and pr; lane q keeps the
    // new pivot row's element of panel column j0 + q
    const int sw = lane + sw0 - j0;  // this lane's column, relative to j0
    T yv = T(0);
    if (sw < jb) {
      T *x = A + (int64_t)col * ld + j0 + sw;
      T *y = A + (int64_t)pr * ld + j0 + sw;
      const T xv = *x;
      yv = *y;
      if (pr != col) {
        *x = yv;
        *y = xv;
      }
    }
    // the lane that swapped panel column j0 + q holds its pivot-row value
    const T prow = __shfl(yv, min(lane + j0 - sw0, WT - 1));
    wave_sync();
    if (!(fabs(pv) > T(0))) flag = 1;
    const T inv = T(1) / pv;
    T pc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) pc[q] = read_lane(prow, q);
    // eliminate below the pivot, two rows per lane per batch
    for (int r0 = col + 1 + lane; r0 < na; r0 += 2 * WT) {
      const int r1 = r0 + WT;
      T *p0 = A + (int64_t)r0 * ld + j0;
      T *p1 = A + (int64_t)r1 * ld + j0;
      const bool h1 = r1 < na;
      T x0[NB], x1[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const bool in = q >= jj && q < jb;
        x0[q] = in ? p0[q] : T(0);
        x1[q] = (in && h1) ? p1[q] : T(0);
      }
      T l0 = T(0), l1 = T(0);
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q == jj) {
          l0 = x0[q] * inv;
          l1 = x1[q] * inv;
        }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (q < jj || q >= jb) continue;
        const T v0 = q == jj ? l0 : fma(-l0, pc[q], x0[q]);
        const T v1 = q == jj ? l1 : fma(-l1, pc[q], x1[q]);
        p0[q] = v0;
        if (h1) p1[q] = v1;
      }
    }
    wave_sync();
  }
  return flag;
}

// The same factorisation with the panel held in registers, for panels of
// at most 256 rows (row j0 + lane + 64 t of the panel in slot t): one load and
// one store of the panel, and per column only cross-lane operations --
// pivot search, the interchange, and the eliminations need no memory round
// trip.  Interchanges swap rows of the panel only.
constexpr int PR_T = 4;  // panel rows per lane
typedef double d16 __attribute__((ext_vector_type(16)));
typedef float fv16 __attribute__((ext_vector_type(16)));
template <class T>
struct V16;
template <>
struct V16<double> {
  typedef d16 t;
};
template <>
struct V16<float> {
  typedef fv16 t;
};

// x0..x3 are four 16-wide row vectors (not an array, which would be placed
// in scratch memory); PR_EACH applies M to each with its slot index.
#define PR_EACH(M) M(0, x0) M(1, x1) M(2, x2) M(3, x3)

template <class T>
__device__ int wave_panel_regs(T *A, int na, int ld, int j0, int jb,
                               int po, WaveLds &W) {
  static_assert(NB == 16, "row vectors hold one 16-column panel");
  typedef typename V16<T>::t vec;
  const int lane = lane_id();
  vec x0, x1, x2, x3;
#define PR_LOAD(t, xv)                                                    \
  {                                                                       \
    const int r = j0 + lane + WT * t;                                     \
    _Pragma("unroll") for (int q = 0; q < NB; ++q) xv[q] =                \
        (r < na && q < jb) ? A[(int64_t)r * ld + j0 + q] : T(0);          \
  }
  PR_EACH(PR_LOAD)
#undef PR_LOAD
  int flag = 0;
#pragma unroll
  for (int jj = 0; jj < NB; ++jj) {
    if (jj < jb) {  // uniform; the loop is unrolled so jj is a constant
      const int col = j0 + jj;
      T ba = T(-1), bv = T(0);
      int bi = na;
#define PR_ARGMAX(t, xv)                                                  \
  {                                                                       \
    const int r = j0 + lane + WT * t;                                     \
    const T v = xv[jj];                                                   \
    if (r >= col && r < na && fabs(v) > ba) {                             \
      ba = fabs(v);                                                       \
      bv = v;                                                             \
      bi = r;                                                             \
    }                                                                     \
  }
      PR_EACH(PR_ARGMAX)
#undef PR_ARGMAX
      wave_argmax(ba, bv, bi);
      int pr = __builtin_amdgcn_readfirstlane(bi);
      const bool bad = pr >= na;  // every candidate is NaN
      if (bad) pr = col;
      if (lane == 0) W.piv[po + jj] = pr;
      const int d = pr - j0;
      const int lp = __builtin_amdgcn_readfirstlane(d & (WT - 1)), tp = d >> 6;
      const bool swap = pr != col, on_p = lane == lp, on_c = lane == jj;
      vec pc;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const T s = tp == 0 ? x0[q] : tp == 1 ? x1[q] : tp == 2 ? x2[q] : x3[q];
        const T vp = read_lane(s, lp);      // pivot row
        const T vc = read_lane((T)x0[q], jj);  // row col (lane jj, slot 0)
        pc[q] = vp;
        // branch-free: the pivot row's slot takes row col, lane jj's slot 0
        // takes the pivot row
        const bool wp = swap && on_p;
        x0[q] = (swap && on_c) ? vp : (wp && tp == 0) ? vc : x0[q];
        x1[q] = (wp && tp == 1) ? vc : x1[q];
        x2[q] = (wp && tp == 2) ? vc : x2[q];
        x3[q] = (wp && tp == 3) ? vc : x3[q];
      }
      const T pv = bad ? (T)__builtin_nan("") : (T)pc[jj];
      if (!(fabs(pv) > T(0))) flag = 1;
      const T inv = T(1) / pv;
#define PR_ELIM(t, xv)                                                    \
  {                                                                       \
    const int r = j0 + lane + WT * t;                                     \
    if (r > col && r < na) {                                              \
      const T l = xv[jj] * inv;                                           \
      xv[jj] = l;                                                         \
      _Pragma("unroll") for (int q = jj + 1; q < NB; ++q) xv[q] =         \
          fma(-l, pc[q], xv[q]);                                          \
    }                                                                     \
  }
      PR_EACH(PR_ELIM)
#undef PR_ELIM
    }
  }
#define PR_STORE(t, xv)                                                   \
  {                                                                       \
    const int r = j0 + lane + WT * t;                                     \
    _Pragma("unroll") for (int q = 0; q < NB; ++q) if (r < na && q < jb)  \
        A[(int64_t)r * ld + j0 + q] = xv[q];                              \
  }
  PR_EACH(PR_STORE)
#undef PR_STORE
  wave_sync();
  return flag;
}
#undef PR_EACH

// Apply the row moves in W (block positions j0 .. j0+cnt-1) to columns
// [c0, c1) only, with batched loads before stores.
template <class T>
__device__ void wave_apply_moves(T *A, int ld, int j0, int cnt, int c0,
                                 int c1, const WaveLds &W) {
  const int lane = lane_id();
  const int nout = W.nout;
  for (int c = c0 + lane; c < c1; c += WT) {
    T xv[NB], yv[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      xv[q] = q < cnt ? A[(int64_t)W.srcp[q] * ld + c] : T(0);
      yv[q] = q < nout ? A[(int64_t)W.osrc[q] * ld + c] : T(0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      if (q < cnt) A[(int64_t)(j0 + q) * ld + c] = xv[q];
      if (q < nout) A[(int64_t)W.opos[q] * ld + c] = yv[q];
    }
  }
  wave_sync();
}

// Invert the NT x NT diagonal block held in W.T into W.Ti (lanes 0..NT-1
// each form one column of the inverse).  Kinds: unit lower triangle (L11 of
// the LU), upper triangle with its diagonal (U11), lower triangle with its
// diagonal (a Cholesky factor).  Padded rows and columns must hold the
// identity.
enum TileKind { TILE_UNIT_LOWER = 0, TILE_UPPER = 1, TILE_LOWER = 2 };
template <int NT>
__device__ void wave_tile_invert(WaveLds &W, int kind) {
  static_assert(NT == 16 || NT == 32, "16 or 32");
  const int lane = lane_id();
  const int j = lane;  // column of the inverse formed by this lane
  // the column in registers (two 16-wide vectors, constant indices only);
  // the block's entries are LDS broadcasts independent of the recurrence
  d16 xa = (d16)0.0, xb = (d16)0.0;
#define TI_GET(q) ((q) < 16 ? xa[(q) & 15] : xb[(q) & 15])
#define TI_SET(q, v)      \
  if ((q) < 16)           \
    xa[(q) & 15] = (v);   \
  else                    \
    xb[(q) & 15] = (v);
  if (kind != TILE_UPPER) {
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      double acc = q == j ? 1.0 : 0.0;
#pragma unroll
      for (int p = 0; p < q; ++p) acc = fma(-W.T[q][p], TI_GET(p), acc);
      if (kind == TILE_LOWER) acc /= W.T[q][q];
      TI_SET(q, acc);
    }
  } else {
#pragma unroll
    for (int q = NT - 1; q >= 0; --q) {
      double acc = q == j ? 1.0 : 0.0;
#pragma unroll
      for (int p = q + 1; p < NT; ++p) acc = fma(-W.T[q][p], TI_GET(p), acc);
      TI_SET(q, acc / W.T[q][q]);
    }
  }
  if (lane < NT) {
#pragma unroll
    for (int q = 0; q < NT; ++q) W.Ti[q][j] = TI_GET(q);
  }
#undef TI_GET
#undef TI_SET
  wave_sync();
}

// Stage the block's diagonal part of A (rows and columns [j0, j0 + jb)) into
// W.T with identity padding to NT: its unit lower triangle (lower) or its
// upper triangle with the diagonal.
template <int NT, class T>
__device__ void wave_tile_stage(const T *A, int ld, int j0, int jb,
                                WaveLds &W, int kind) {
  const int lane = lane_id();
  for (int q = lane; q < NT * NT; q += WT) {
    const int i = q / NT, j = q % NT;
    double v = i == j ? 1.0 : 0.0;
    const bool in = kind == TILE_UNIT_LOWER ? j < i
                    : kind == TILE_UPPER    ? j >= i
                                            : j <= i;
    if (i < jb && j < jb && in) v = (double)A[(int64_t)(j0 + i) * ld + j0 + j];
    W.T[i][j] = v;
  }
  wave_sync();
}

// Row moves of the cnt interchanges W.piv[po + q] at positions j0 + q
// (they act in sequence; a position, once passed, is never moved again):
// W.srcp, W.opos, W.osrc, W.nout.  Lane 0 only.
__device__ void wave_build_moves(WaveLds &W, int j0, int cnt, int po = 0) {
  if (lane_id() == 0) {
    int nout = 0;
    for (int q = 0; q < cnt; ++q) W.srcp[q] = j0 + q;
    for (int q = 0; q < cnt; ++q) {
      const int p = W.piv[po + q];
      if (p == j0 + q) continue;
      int *slot;
      if (p < j0 + cnt) {
        slot = &W.srcp[p - j0];
      } else {
        int m = 0;
        while (m < nout && W.opos[m] != p) ++m;
        if (m == nout) {
          W.opos[m] = p;
          W.osrc[m] = p;
          ++nout;
        }
        slot = &W.osrc[m];
      }
      const int t = W.srcp[q];
      W.srcp[q] = *slot;
      *slot = t;
    }
    W.nout = nout;
  }
  wave_sync();
}

// Columns [c0, c1) of rows j0 .. j0+NT-1:  X <- Ti X (or Ti^T X), where row q of X is
// taken from row srcp[q] (moves) or row j0 + q, and rows opos[m] receive
// rows osrc[m] (m < nout) in the same pass; only rows q < jb are written.
// 16 x 16 FP64 MFMA blocks over NT/4 k-steps; every load of a batch is
// issued before any store, so sources and destinations may coincide.
template <int NT, bool TRANS = false, class T = double>
__device__ void wave_tile_apply(T *A, int ld, int j0, int jb, int c0,
                                int c1, const WaveLds &W, bool moves) {
  constexpr int NS = NT / 4, NRB = NT / 16, CB = NT == 16 ? 4 : 2;
  typedef typename Mx<T>::acc acc_t;
  const int lane = lane_id();
  const int col = lane & 15, kq = lane >> 4;
  T ainv[NRB][NS];  // Ti, or its transpose
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
    for (int s = 0; s < NS; ++s)
      ainv[rb][s] = (T)(TRANS ? W.Ti[4 * s + kq][rb * 16 + col]
                              : W.Ti[rb * 16 + col][4 * s + kq]);
  int srow[NS], orow[NS], drow[NS];
  bool sv[NS], ov[NS];
  const int nout = moves ? W.nout : 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int q = 4 * s + kq;
    sv[s] = q < jb;
    srow[s] = moves ? (sv[s] ? W.srcp[q] : 0) : j0 + q;
    ov[s] = q < nout;
    orow[s] = ov[s] ? W.osrc[q] : 0;
    drow[s] = ov[s] ? W.opos[q] : 0;
  }
  for (int cb = c0; cb < c1; cb += 16 * CB) {
    T b[CB][NS], y[CB][NS];
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      const int c = cb + 16 * u + col;
      const bool cv = c < c1;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        b[u][s] = (cv && sv[s]) ? A[(int64_t)srow[s] * ld + c] : T(0);
        y[u][s] = (cv && ov[s]) ? A[(int64_t)orow[s] * ld + c] : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      acc_t acc[NRB];
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) acc[rb] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
          acc[rb] = Mx<T>::mfma(ainv[rb][s], b[u][s], acc[rb]);
      const int c = cb + 16 * u + col;
      if (c < c1) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (ov[s]) A[(int64_t)drow[s] * ld + c] = y[u][s];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int q = rb * 16 + Mx<T>::row(kq, r);  // result row
            if (q < jb) A[(int64_t)(j0 + q) * ld + c] = acc[rb][r];
          }
      }
    }
  }
  wave_sync();
}

// Solve A X = B in place for the na x na matrix in columns [0, na) of rows
// [0, na) (leading dimension ld), right-hand sides in columns
// [na, na + nrhs); on return those columns hold X.  Wavefront-local.
// Blocks of 32 columns: two 16-column panels (the second updated by the
// first before it is factored), then the block's interchanges and L11^-1
// applied to the columns on its right and one rank-32 trailing update, so
// the trailing matrix crosses HBM once per 32 columns.  Returns nonzero if
// a pivot was zero or not a number.  piv (nullable) receives the pivot row
// of every column, block by block, for later solves with the factors
// (wave_lu_resolve).
// (TAG only makes a separate copy of the routine for a caller in another
// kernel, so that the two kernels' register allocations stay independent.)
template <class T, int TAG = 0>
__device__ int wave_lu_solve(T *A, int na, int ld, int nrhs, WaveLds &W,
                             int *piv = nullptr) {
  const int ntot = na + nrhs;
  int flag = 0;
  for (int j0 = 0; j0 < na; j0 += NB2) {
    const int jb = min(NB2, na - j0);
    const int ja = min(NB, jb);
    const bool regs = na - j0 <= PR_T * WT;
    flag |= regs ? wave_panel_regs(A, na, ld, j0, ja, 0, W)
                 : wave_panel(A, na, ld, j0, ja, j0, 0, W);
    if (jb > ja) {
      // first panel's interchanges and L^-1 on the second panel's columns,
      // then its update of the second panel's rows below
      wave_build_moves(W, j0, ja);
      wave_tile_stage<NB>(A, ld, j0, ja, W, TILE_UNIT_LOWER);
      wave_tile_invert<NB>(W, TILE_UNIT_LOWER);
      wave_tile_apply<NB>(A, ld, j0, ja, j0 + ja, j0 + jb, W, true);
      wave_gemm<0>(A + (int64_t)(j0 + ja) * ld + j0 + ja, ld,
                   A + (int64_t)(j0 + ja) * ld + j0, ld,
                   A + (int64_t)j0 * ld + j0 + ja, ld, na - j0 - ja, jb - ja,
                   ja);
      if (regs) {
        // the second panel's interchanges also move the first panel's L
        flag |= wave_panel_regs(A, na, ld, j0 + ja, jb - ja, ja, W);
        wave_build_moves(W, j0 + ja, jb - ja, ja);
        wave_apply_moves(A, ld, j0 + ja, jb - ja, j0, j0 + ja, W);
      } else {
        flag |= wave_panel(A, na, ld, j0 + ja, jb - ja, j0, ja, W);
      }
    }
    // the block's interchanges and L11^-1 on every column to its right
    if (piv && lane_id() < jb) piv[j0 + lane_id()] = W.piv[lane_id()];
    wave_build_moves(W, j0, jb);
    wave_tile_stage<NB2>(A, ld, j0, jb, W, TILE_UNIT_LOWER);
    wave_tile_invert<NB2>(W, TILE_UNIT_LOWER);
    wave_tile_apply<NB2>(A, ld, j0, jb, j0 + jb, ntot, W, true);
    const int r0 = j0 + jb;
    if (r0 < na)
      wave_gemm_wide<0, 0, 2, 4>(A + (int64_t)r0 * ld + r0, ld,
                                 A + (int64_t)r0 * ld + j0, ld,
                                 A + (int64_t)j0 * ld + r0, ld, na - r0,
                                 ntot - r0, jb);
  }
  // back substitution U X = B' on the right-hand sides, 32 rows at a time
  for (int j0 = ((na - 1) / NB2) * NB2; j0 >= 0; j0 -= NB2) {
    const int jb = min(NB2, na - j0);
    const int r1 = j0 + jb;
    // left-looking: this block's rows take the solved rows below at once
    // (X_b -= U[b, >b] X[>b]), so the right-hand sides above are not
    // rewritten once per block
    if (r1 < na)
      wave_gemm_wide<0, 0, 2, 4>(A + (int64_t)j0 * ld + na, ld,
                                 A + (int64_t)j0 * ld + r1, ld,
                                 A + (int64_t)r1 * ld + na, ld, jb, nrhs,
                                 na - r1);
    wave_tile_stage<NB2>(A, ld, j0, jb, W, TILE_UPPER);
    wave_tile_invert<NB2>(W, TILE_UPPER);
    wave_tile_apply<NB2>(A, ld, j0, jb, na, ntot, W, false);
  }
  return flag;
}

// Solve A X = B again with the factors wave_lu_solve left in columns
// [0, na) and its pivots `piv`, for new right-hand sides in columns
// [na, na + nrhs); on return those columns hold X.  Same block order as the
// factorisation: per 32-column block its interchanges and L11^-1 on the
// right-hand sides, then the rank-32 update of the rows below (the L
// columns of a block were never permuted by later blocks, so they match the
// right-hand sides at that point), then back substitution with U.
template <class T>
__device__ void wave_lu_resolve(T *A, int na, int ld, int nrhs,
                                const int *piv, WaveLds &W) {
  const int lane = lane_id();
  const int ntot = na + nrhs;
  for (int j0 = 0; j0 < na; j0 += NB2) {
    const int jb = min(NB2, na - j0);
    if (lane < jb) W.piv[lane] = piv[j0 + lane];
    wave_sync();
    wave_build_moves(W, j0, jb);
    wave_tile_stage<NB2>(A, ld, j0, jb, W, TILE_UNIT_LOWER);
    wave_tile_invert<NB2>(W, TILE_UNIT_LOWER);
    wave_tile_apply<NB2>(A, ld, j0, jb, na, ntot, W, true);
    const int r0 = j0 + jb;
    if (r0 < na)
      wave_gemm_wide<0, 0, 2, 4>(A + (int64_t)r0 * ld + na, ld,
                                 A + (int64_t)r0 * ld + j0, ld,
                                 A + (int64_t)j0 * ld + na, ld, na - r0, nrhs,
                                 jb);
  }
  for (int j0 = ((na - 1) / NB2) * NB2; j0 >= 0; j0 -= NB2) {
    const int jb = min(NB2, na - j0);
    const int r1 = j0 + jb;
    // left-looking: this block's rows take the solved rows below at once
    // (X_b -= U[b, >b] X[>b]), so the right-hand sides above are not
    // rewritten once per block
    if (r1 < na)
      wave_gemm_wide<0, 0, 2, 4>(A + (int64_t)j0 * ld + na, ld,
                                 A + (int64_t)j0 * ld + r1, ld,
                                 A + (int64_t)r1 * ld + na, ld, jb, nrhs,
                                 na - r1);
    wave_tile_stage<NB2>(A, ld, j0, jb, W, TILE_UPPER);
    wave_tile_invert<NB2>(W, TILE_UPPER);
    wave_tile_apply<NB2>(A, ld, j0, jb, na, ntot, W, false);
  }
}

// Residual of the matching system in FP64 for iterative refinement.  With R
// (n x n, leading dimension ld) and the current solution Z (n x no, ld),
//   B - M Z = R (D2 Z + E) - [diag(s); 0] - D1 Z,   E_kj = a s'_j [k == j],
// from the channel slots (d1, d2, s, a s'), so neither M nor B is kept.  R W
// runs as 16x16x4 FP64 MFMAs over 32 x 32 output tiles with W formed in the
// fragment loads; the residual goes to `out` (FP32, leading dimension ldo).
// Returns max |r| (wavefront-uniform).
__device__ double wave_residual(const double *Rm, int ld, const double *Z,
                                const ChanSlot *ch, int n, int no,
                                float *out, int ldo) {
  const int lane = lane_id();
  const int col = lane & 15, kq = lane >> 4;
  const int nct = (no + 31) >> 5, ntile = ((n + 31) >> 5) * nct;
  double rmax = 0.0;
  for (int t = 0; t < ntile; ++t) {
    const int rb = (t / nct) * 32, cb = (t % nct) * 32;
    d4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += 16) {
      double a[4][2], b[4][2];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = k0 + 4 * s4 + kq;
        const bool kv = k < n;
        const double d2 = kv ? ch[k].d2 : 0.0;
        const double asp = kv ? ch[k].asp : 0.0;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const int i = rb + 16 * x + col;
          a[s4][x] = (kv && i < n) ? Rm[(int64_t)i * ld + k] : 0.0;
          const int j = cb + 16 * x + col;
          const double z = (kv && j < no) ? Z[(int64_t)k * ld + j] : 0.0;
          b[s4][x] = (kv && j < no) ? fma(d2, z, k == j ? asp : 0.0) : 0.0;
        }
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                a[s4][x], b[s4][y], acc[x][y], 0, 0, 0);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rb + 16 * x + kq + 4 * r, j = cb + 16 * y + col;
          if (i >= n || j >= no) continue;
          const double z = Z[(int64_t)i * ld + j];
          double v = acc[x][y][r] - ch[i].d1 * z;
          if (i == j) v -= ch[i].s;
          rmax = fmax(rmax, fabs(v));
          out[(int64_t)i * ldo + j] = (float)v;
        }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, off));
  wave_sync();
  return rmax;
}

// Copy a rows x cols block (row-major source ld sl, destination ld dl) with
// batched loads.
__device__ inline void wave_copy(double *dst, int dl, const double *src,
                                 int sl, int rows, int cols) {
  const int lane = lane_id();
  const int nq = rows * cols;
  for (int q0 = lane; q0 < nq; q0 += UNR * WT) {
    double v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      v[u] = q < nq ? src[(int64_t)(q / cols) * sl + q % cols] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      if (q < nq) dst[(int64_t)(q / cols) * dl + q % cols] = v[u];
    }
  }
}

// ---------------------------------------------------------------------------
// T step by Cholesky.  T = 2iK (1 - iK)^-1 = 2(1 - iK)^-1 - 2 and
// (1 - iK)^-1 = (1 + iK)(1 + K^2)^-1, so with A = (1 + K^2)^-1 (K, A and
// K A are symmetric and commute)
//     Re T = -2 Q,  Q = K^2 A = 1 - A,     Im T = 2 Y,  Y = K A,
// and |T_ij|^2 = 4 (Y_ij^2 + Q_ij^2).  1 + K^2 is symmetric positive
// definite (eigenvalues 1 + k^2 >= 1): no pivoting, only its lower triangle
// is formed and factored, 1 + K^2 = L L^T.  A = L^-T L^-1 from the lower
// triangular L^-1 (forward substitution on the identity, each block only
// on the columns left of its end) and a product that starts each tile's sum
// at its first row; Y = K A with A read from its lower triangle.  That is
// (1 + 1/3 + 1/3 + 1/3 + 1) no^3 flops with the product 1 + K^2; the route
// Z = L^-1 K, Q = Z^T Z, Y = L^-T Z takes (1 + 1/3 + 1 + 1 + 1) no^3.
// Off the diagonal Q = -A exactly; on it Q_ii = 1 - A_ii, whose absolute
// error (unit roundoff) matters only where Q_ii itself is that small.
// Forming 1 + K^2 squares the condition number of 1 - iK, and the product
// K A multiplies the rounding of A by |K|: this route's error grows as the
// square of K's largest row norm (about 3e-17 |K|_row^2 against the exact
// T, 1e-8 at 1e4, 3e-2 at 2.5e7, which a 1e5-point mesh reaches where an
// eigenphase is within ~1e-8 of pi/2).  Energies where 1 + K^2 has a
// diagonal entry (1 + that row norm squared) above kTInvMax instead solve
// (1 - iK) W = 1 directly, as the real system
//     [ 1  K ] [X]   [1]
//     [-K  1 ] [Y] = [0],    W = X + iY,  X = A,  Y = K A,
// by the wavefront LU with partial pivoting: its condition number is that
// of 1 - iK, about |K|, so the error stays near u |K| (6e-10 at 7e7 in an
// FP64 emulation).  That takes a slot of 6 n^2 doubles from the launch's
// pool; without one the energy takes the route through Z = L^-1 K
// (Q = Z^T Z, Y = L^-T Z), whose error grows more slowly than the A route's
// but still with |K|^2; the latter also serves when every slot of the
// complex route's buffer pool is taken.  At 200 channels about 0.5 % of a
// uniform mesh's energies are above the threshold.
constexpr double kTInvMax = 1e8;
enum TRoute { T_ROUTE_A = 0, T_ROUTE_Z = 1 };

// Factor the jb x jb (jb <= 32) diagonal block at (j0, j0) of A = L L^T in
// registers: lane i holds row i in two 16-wide vectors; per column, one
// broadcast of the diagonal and of the column, no memory round trip.
// Writes L11 back (lower triangle with its diagonal) and stages it in W.T
// for inversion.  Returns 1 if a diagonal was not positive.
__device__ int wave_chol_diag(double *A, int ld, int j0, int jb, WaveLds &W) {
  const int lane = lane_id();
  d16 xa, xb;  // row `lane`, columns 0..15 and 16..31 of the block
  const bool row_ok = lane < jb;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    xa[k] = (row_ok && k <= lane) ? A[(int64_t)(j0 + lane) * ld + j0 + k] : 0.0;
    xb[k] = (row_ok && 16 + k <= lane && 16 + k < jb)
                ? A[(int64_t)(j0 + lane) * ld + j0 + 16 + k]
                : 0.0;
  }
  int flag = 0;
#define CH_GET(j) ((j) < 16 ? xa[(j) & 15] : xb[(j) & 15])
#define CH_SET(j, v)          \
  if ((j) < 16)               \
    xa[(j) & 15] = (v);       \
  else                        \
    xb[(j) & 15] = (v);
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    if (j < jb) {  // uniform; the loop is unrolled so j is a constant
      const double djj = read_lane(CH_GET(j), j);
      if (!(djj > 0.0)) flag = 1;
      const double d = sqrt(djj), rd = 1.0 / d;
      const double lij = lane > j ? CH_GET(j) * rd : lane == j ? d : CH_GET(j);
      CH_SET(j, lij);
#pragma unroll
      for (int k = j + 1; k < 32; ++k) {
        if (k < jb) {
          const double lkj = read_lane(lij, k);  // L[k][j]
          const double v = CH_GET(k);
          CH_SET(k, lane >= k ? fma(-lij, lkj, v) : v);
        }
      }
    }
  }
#undef CH_GET
#undef CH_SET
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if (row_ok && k <= lane) A[(int64_t)(j0 + lane) * ld + j0 + k] = xa[k];
    if (row_ok && 16 + k <= lane && 16 + k < jb)
      A[(int64_t)(j0 + lane) * ld + j0 + 16 + k] = xb[k];
  }
  // W.T: the factor with identity padding
  if (lane < NB2) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      W.T[lane][k] = row_ok ? (k <= lane ? xa[k] : 0.0) : (k == lane ? 1.0 : 0.0);
      W.T[lane][16 + k] = row_ok ? (16 + k <= lane ? xb[k] : 0.0)
                                 : (16 + k == lane ? 1.0 : 0.0);
    }
  }
  wave_sync();
  return flag;
}

// Rows [r0, r1) of columns [j0, j0 + jb): X <- X Ti^T (the panel of a
// Cholesky factor, L21 = A21 L11^-T), 16 rows at a time as FP64 MFMA
// blocks; each row block is loaded whole before it is stored.
__device__ void wave_rows_times_tit(double *A, int ld, int r0, int r1, int j0,
                                    int jb, const WaveLds &W) {
  const int lane = lane_id();
  const int col = lane & 15, kq = lane >> 4;
  double b[2][8];  // B[k][j] = Ti[j][k], j = 16 cb + col, k = 4 s + kq
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int s = 0; s < 8; ++s) b[cb][s] = W.Ti[16 * cb + col][4 * s + kq];
  for (int rb = r0; rb < r1; rb += 32) {
    double a[2][8];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = rb + 16 * h + col;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int k = 4 * s + kq;
        a[h][s] = (r < r1 && k < jb) ? A[(int64_t)r * ld + j0 + k] : 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      d4 acc[2];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h][s], b[cb][s],
                                                         acc[cb], 0, 0, 0);
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rb + 16 * h + kq + 4 * r, j = 16 * cb + col;
          if (row < r1 && j < jb) A[(int64_t)row * ld + j0 + j] = acc[cb][r];
        }
    }
  }
  wave_sync();
}

// The T step in the workspace of one energy: K (no x no, leading dimension
// lk) in; Y in columns [no, 2 no) of Aug (leading dimension ld) and the
// lower triangle of Q in K's place out; Aug's columns [0, no) hold L.  Returns nonzero if 1 + K^2 was
// not positive definite in floating point.
// Photoionization: one block step of the forward substitution y = L^-1 v
// of the dipole amplitudes v (no entries, global memory), with Ti = L11^-1
// of the block in W: y_b = Ti v_b, then v[r] -= L[r][b] y_b below it.  y_b
// is broadcast through the first row of W.T, free once Ti is formed.
__device__ void wave_photo_forward(const double *Aug, int ld, int j0, int jb,
                                   int no, WaveLds &W, double *v) {
  const int lane = lane_id();
  const double vb = lane < jb ? v[j0 + lane] : 0.0;
  double y = 0.0;
#pragma unroll
  for (int k = 0; k < NB2; ++k)
    y = fma(W.Ti[lane & (NB2 - 1)][k], read_lane(vb, k), y);
  y = lane < jb ? y : 0.0;
  if (lane < NB2) W.T[0][lane] = y;
  if (lane < jb) v[j0 + lane] = y;
  wave_sync();
  for (int r = j0 + jb + lane; r < no; r += WT) {
    const double *Lr = Aug + (int64_t)r * ld + j0;
    double acc = v[r];
#pragma unroll
    for (int k0 = 0; k0 < NB2; k0 += 8) {
      double lv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) lv[k] = k0 + k < jb ? Lr[k0 + k] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) acc = fma(-lv[k], W.T[0][k0 + k], acc);
    }
    v[r] = acc;
  }
  wave_sync();
}

// The T step's route for large K: (1 - iK) W = 1 as the real system
// [1 K; -K 1] [X; Y] = [1; 0] in `ext` (2 no x 3 no, leading dimension
// 3 no), solved by the wavefront LU; X into Aug's columns [0, no), Y into
// [no, 2 no).  Kept out of line: it runs at few energies, and inlined it
// would raise the register pressure of the whole matching kernel.
__device__ __attribute__((noinline)) int wave_t_complex(
    double *Aug, int ld, const double *Kb, int lk, int no, double *ext,
    WaveLds &W) {
  const int lane = lane_id();
  // [1 K | 1; -K 1 | 0], leading dimension 3 no, solved in place
  const int l3 = 3 * no, nq = 2 * no * l3;
  for (int q0 = lane; q0 < nq; q0 += UNR * WT) {
    double v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      const int i = q / l3, j = q % l3;
      const int ib = i < no ? i : i - no, jb = j % no;
      const int blk = (i < no ? 0 : 3) + j / no;  // 0 1 2 / 3 4 5
      double x = 0.0;
      if (q < nq) {
        if (blk == 1 || blk == 3) x = Kb[(int64_t)ib * lk + jb];
        if (blk == 3) x = -x;
        if ((blk == 0 || blk == 2 || blk == 4) && ib == jb) x = 1.0;
      }
      v[u] = x;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      if (q < nq) ext[(int64_t)(q / l3) * l3 + q % l3] = v[u];
    }
  }
  wave_sync();
  const int flag = wave_lu_solve(ext, 2 * no, l3, no, W) ? 1 : 0;
  // X (rows [0, no)) over 1 + K^2's place, Y (rows [no, 2 no)) beside it
  const int nsq = no * no;
  for (int q0 = lane; q0 < nsq; q0 += UNR * WT) {
    double x[UNR], y[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      const int i = q / no, j = q % no;
      x[u] = q < nsq ? ext[(int64_t)i * l3 + 2 * no + j] : 0.0;
      y[u] = q < nsq ? ext[(int64_t)(no + i) * l3 + 2 * no + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      if (q >= nsq) continue;
      const int i = q / no, j = q % no;
      Aug[(int64_t)i * ld + j] = x[u];
      Aug[(int64_t)i * ld + no + j] = y[u];
    }
  }
  wave_sync();
  return flag;
}

// want_t: form Y and Q or A (collision strengths); pv: dipole amplitudes to
// be replaced by L^-1 pv (photoionization), or null; ext: the workspace's
// complex-system part, or null.  On return with want_t, the lower triangle
// of Y is in columns [no, 2 no) of Aug and `route` says where Q is:
// T_ROUTE_A, A = 1 - Q (lower triangle) in columns [0, no) of Aug and Kb is
// free; T_ROUTE_Z, the lower triangle of Q in Kb and Aug's columns [0, no)
// are free.
__device__ int wave_tstep(double *Aug, int ld, double *Kb, int lk, int no,
                          WaveLds &W, bool want_t, double *pv,
                          const MatchLaunch &L, int e, int &route) {
  int flag = 0;
  const int lane = lane_id();
  // lower triangle of 1 + K^2
  wave_gemm_wide<1, G_LOWER, 2, 4>(Aug, ld, Kb, lk, Kb, lk, no, no, no);
  // route: the largest diagonal entry 1 + sum_j K_ij^2 (wavefront-uniform)
  double gmax = 0.0;
  for (int i = lane; i < no; i += WT) gmax = fmax(gmax, Aug[(int64_t)i * ld + i]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, off));
  const bool inv = gmax <= kTInvMax;
  // a slot of the complex route's pool, taken by lane 0 (the loop is
  // bounded: with every slot taken the energy goes through Z instead)
  int slot = -1;
  if (want_t && !inv && L.ext && t_ext_doubles(no) <= L.ext_estride) {
    if (lane == 0) {
      for (int t = 0; t < L.ext_slots; ++t) {
        const int q = (e + t) % L.ext_slots;
        if (atomicCAS(&L.ext_flags[q], 0, 1) == 0) {
          slot = q;
          break;
        }
      }
    }
    slot = __builtin_amdgcn_readfirstlane(slot);
  }
  const bool cplx = slot >= 0;
  double *ext = cplx ? L.ext + (int64_t)slot * L.ext_estride : nullptr;
  const bool rhs = want_t && !cplx;
  route = (inv || cplx) ? T_ROUTE_A : T_ROUTE_Z;
  // right-hand side: the identity (route through A) or K (route through Z)
  if (rhs && inv) {
    const int nsq = no * no;
    for (int q = lane; q < nsq; q += WT) {
      const int i = q / no, j = q % no;
      Aug[(int64_t)i * ld + no + j] = i == j ? 1.0 : 0.0;
    }
  } else if (rhs) {
    wave_copy(Aug + no, ld, Kb, lk, no, no);
  }
  wave_sync();
  // right-looking blocked Cholesky with the forward substitution; with the
  // identity, rows of block b have nonzeros only left of the block's end
  if (pv || rhs) {
    for (int j0 = 0; j0 < no; j0 += NB2) {
      const int jb = min(NB2, no - j0);
      flag |= wave_chol_diag(Aug, ld, j0, jb, W);
      wave_tile_invert<NB2>(W, TILE_LOWER);
      const int r0 = j0 + jb;
      const int rc = inv ? r0 : no;  // right-hand-side columns in play
      if (r0 < no) wave_rows_times_tit(Aug, ld, r0, no, j0, jb, W);
      if (pv) wave_photo_forward(Aug, ld, j0, jb, no, W, pv);
      if (rhs) wave_tile_apply<NB2>(Aug, ld, j0, jb, no, no + rc, W, false);
      if (r0 < no) {
        wave_gemm_wide<0, G_TB | G_LOWER, 2, 4>(
            Aug + (int64_t)r0 * ld + r0, ld, Aug + (int64_t)r0 * ld + j0, ld,
            Aug + (int64_t)r0 * ld + j0, ld, no - r0, no - r0, jb);
        if (rhs)
          wave_gemm_wide<0, 0, 2, 4>(Aug + (int64_t)r0 * ld + no, ld,
                                     Aug + (int64_t)r0 * ld + j0, ld,
                                     Aug + (int64_t)j0 * ld + no, ld, no - r0,
                                     rc, jb);
      }
    }
  }
  if (!want_t) return flag;
  if (cplx) {
    flag |= wave_t_complex(Aug, ld, Kb, lk, no, ext, W);
    // every read of the slot is done (its values were stored into Aug)
    // before the slot is given back
    __threadfence();
    if (lane == 0) atomicExch(&L.ext_flags[slot], 0);
    return flag;
  }
  if (inv) {
    // A = (L^-1)^T L^-1, lower triangle, over L's place
    wave_gemm_wide<2, G_TA | G_LOWER | G_KTRI, 2, 4>(Aug, ld, Aug + no, ld,
                                                     Aug + no, ld, no, no, no);
    // Y = K A, lower triangle, over L^-1's place
    wave_gemm_wide<2, G_BSYM | G_LOWER, 2, 4>(Aug + no, ld, Kb, lk, Aug, ld,
                                              no, no, no);
    return flag;
  }
  // Q = Z^T Z (= K^2 A) in K's place, lower triangle
  wave_gemm_wide<2, G_TA | G_LOWER, 2, 4>(Kb, lk, Aug + no, ld, Aug + no, ld,
                                          no, no, no);
  // Y = L^-T Z, blocks from the bottom
  for (int j0 = ((no - 1) / NB2) * NB2; j0 >= 0; j0 -= NB2) {
    const int jb = min(NB2, no - j0);
    const int r1 = j0 + jb;
    // left-looking, as the LU's back substitution: Z_b -= L[>b, b]^T Y[>b]
    if (r1 < no)
      wave_gemm_wide<0, G_TA, 2, 4>(Aug + (int64_t)j0 * ld + no, ld,
                                    Aug + (int64_t)r1 * ld + j0, ld,
                                    Aug + (int64_t)r1 * ld + no, ld, jb, no,
                                    no - r1);
    wave_tile_stage<NB2>(Aug, ld, j0, jb, W, TILE_LOWER);
    wave_tile_invert<NB2>(W, TILE_LOWER);
    wave_tile_apply<NB2, true>(Aug, ld, j0, jb, no, 2 * no, W, false);
  }
  return flag;
}

// ---------------------------------------------------------------------------
// Collision strengths.
//
// V_ij = Y_ij^2 + Q_ij^2 over the open block; Omega(t, u) += 2g sum_{i in t,
// j in u} V_ij.  When every target level holds one channel the sum is a
// relabelling of V's upper triangle; otherwise it is G^T V G with the 0/1
// channel-to-level matrix G (two MFMA products).

__device__ inline int64_t omega_index(int t, int u, int n_out) {
  if (t > u) {
    const int x = t;
    t = u;
    u = x;
  }
  return (int64_t)t * n_out - ((int64_t)t * (t - 1)) / 2 + (u - t);
}

// Start of row i of the row-major upper triangle of an m x m matrix.
__device__ inline int64_t tri_row_start(int i, int m) {
  return (int64_t)i * m - ((int64_t)i * (i - 1)) / 2;
}

// Row i and column j >= i of entry p of that triangle.
__device__ inline void tri_decode(int64_t p, int m, int &i, int &j) {
  const double b = 2.0 * m + 1.0;
  int r = (int)((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
  r = max(0, min(r, m - 1));
  while (r > 0 && tri_row_start(r, m) > p) --r;
  while (r + 1 < m && tri_row_start(r + 1, m) <= p) ++r;
  i = r;
  j = r + (int)(p - tri_row_start(r, m));
}

// The lower triangles of Y (leading dimension ldy) and of Q, or of A with
// Q = 1 - A (q_is_a), in Qm (ldq) over the open block in; V (ldv, disjoint
// from both) is scratch, and so is Qm once V is formed.  Returns 1 if a
// contribution was not finite.
__device__ int wave_omega(const SymDev &S, int n_out, const double *Y, int ldy,
                          double *Qm, int ldq, bool q_is_a, double *V, int ldv,
                          int no, double *om) {
  const int lane = lane_id();
  const double g2 = 2.0 * S.g;
  int nonfinite = 0;
  if (S.ntu == S.n) {
    // one channel per level: walk the open block's upper triangle
    const int64_t npair = (int64_t)no * (no + 1) / 2;
    for (int64_t p0 = lane; p0 < npair; p0 += UNR * WT) {
      int ii[UNR], jj[UNR], ti[UNR], tj[UNR];
      double yv[UNR], qv[UNR], ov[UNR];
      int64_t oi[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int64_t p = p0 + (int64_t)u * WT;
        ii[u] = 0;
        jj[u] = 0;
        if (p < npair) tri_decode(p, no, ii[u], jj[u]);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const bool in = p0 + (int64_t)u * WT < npair;
        ti[u] = in ? S.tgt[ii[u]] : 0;
        tj[u] = in ? S.tgt[jj[u]] : 0;
        // lower triangles: row jj >= column ii
        const double qa = in ? Qm[(int64_t)jj[u] * ldq + ii[u]] : 0.0;
        qv[u] = q_is_a ? (in && ii[u] == jj[u] ? 1.0 : 0.0) - qa : qa;
        yv[u] = in ? Y[(int64_t)jj[u] * ldy + ii[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const bool in = p0 + (int64_t)u * WT < npair;
        oi[u] = omega_index(ti[u], tj[u], n_out);
        ov[u] = in ? om[oi[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        if (p0 + (int64_t)u * WT >= npair) continue;
        const double v = g2 * (yv[u] * yv[u] + qv[u] * qv[u]);
        if (!isfinite(v)) nonfinite = 1;
        om[oi[u]] = ov[u] + v;
      }
    }
    return nonfinite;
  }
  // V, both triangles
  const int nsq = no * no;
  for (int q0 = lane; q0 < nsq; q0 += UNR * WT) {
    double yv[UNR], qv[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      const int qi = q / no, qj = q % no;
      const int64_t lo = (int64_t)max(qi, qj), co = min(qi, qj);
      const double qa = q < nsq ? Qm[lo * ldq + co] : 0.0;
      qv[u] = q_is_a ? (q < nsq && qi == qj ? 1.0 : 0.0) - qa : qa;
      yv[u] = q < nsq ? Y[lo * ldy + co] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      if (q < nsq)
        V[(int64_t)(q / no) * ldv + q % no] = yv[u] * yv[u] + qv[u] * qv[u];
    }
  }
  wave_sync();
  const int nt = S.ntu;
  // W1 = G^T V (nt x no) into Qm's place, then Omega_u = W1 G (nt x nt) into V
  wave_gemm<2>(Qm, ldq, S.GT, S.n, V, ldv, nt, no, no);
  wave_gemm<2>(V, ldv, Qm, ldq, S.G, nt, nt, nt, no);
  const int64_t npair = (int64_t)nt * (nt + 1) / 2;
  for (int64_t p0 = lane; p0 < npair; p0 += UNR * WT) {
    int ta[UNR], tb[UNR];
    double v[UNR], ov[UNR];
    int64_t oi[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int64_t p = p0 + (int64_t)u * WT;
      ta[u] = 0;
      tb[u] = 0;
      if (p < npair) tri_decode(p, nt, ta[u], tb[u]);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const bool in = p0 + (int64_t)u * WT < npair;
      v[u] = in ? V[(int64_t)ta[u] * ldv + tb[u]] : 0.0;
      const int t = in ? S.ut[ta[u]] : 0, w = in ? S.ut[tb[u]] : 0;
      oi[u] = omega_index(t, w, n_out);
      ov[u] = in ? om[oi[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      if (p0 + (int64_t)u * WT >= npair) continue;
      const double c = g2 * v[u];
      if (!isfinite(c)) nonfinite = 1;
      om[oi[u]] = ov[u] + c;
    }
  }
  return nonfinite;
}

// ---------------------------------------------------------------------------

// Channel functions of symmetry S at energy Ee into ch[0..n), sorted order.
__device__ int wave_channel_functions(const SymDev &S, double Ee,
                                      ChanSlot *ch) {
  const int lane = lane_id();
  int bits = 0;
  const double ra = S.r_match;
  for (int i = lane; i < S.n; i += WT) {
    const double diff = Ee - S.e_thr[i];
    ChanSlot c;
    if (diff > 0.0) {
      const OpenVals v = coulomb_open(S.l[i], S.z, sqrt(diff), ra);
      c.d1 = v.c;
      c.d2 = ra * v.cp;
      c.s = v.s;
      c.asp = ra * v.sp;
      if (!v.ok) bits |= RM_E_CF_NOCONV;
    } else if (diff < 0.0) {
      const ClosedVals v = whittaker_closed(S.l[i], S.z, sqrt(-diff), ra);
      c.d1 = v.e;
      c.d2 = v.ep;
      c.s = 0.0;
      c.asp = 0.0;
      if (!v.ok) bits |= RM_E_CF_NOCONV;
    } else {
      c.d1 = 1.0;
      c.d2 = 0.0;
      c.s = 0.0;
      c.asp = 0.0;
      bits |= RM_E_ON_THRESHOLD;
    }
    ch[i] = c;
  }
  return bits;
}

__device__ inline int count_open(const SymDev &S, double Ee) {
  int lo = 0, hi = S.n;  // thresholds strictly below E
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (S.e_thr[mid] < Ee)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// The matching solve with an FP32 factorisation refined in FP64: [M | B]
// rounded to FP32 in K's place (n x 2n floats), factored and solved there;
// the solution Z in FP64 in Aug's right half, then per iteration the FP64
// residual (wave_residual, from R kept in Aug's left half) solved with the
// FP32 factors and added to Z.  Converged when a correction is below the
// rounding of Z (max|dZ| <= 2^-50 max|Z|), or when the corrections stop
// contracting (max|dZ| over half the previous one) at a residual that passes
// the backward-error test of LAPACK's mixed-precision dsgesv, max|r| <=
// 4 sqrt(n) u ||M||_inf max|Z| (u = 2^-53): the floor that the system's
// conditioning sets in FP64.  Otherwise, after refine_iters corrections,
// the energy is flagged RM_E_REFINE_NOCONV and solved again with the FP64
// factorisation.  Returns RM_E_* bits.
__device__ int wave_solve_fp32(const MatchLaunch &L, const SymDev &S,
                               double *Aug, double *Kb, const ChanSlot *ch,
                               int no, WaveLds &W) {
  const int lane = lane_id();
  const int n = S.n, ld = 2 * n, ld32 = 2 * n;
  float *A32 = (float *)Kb;
  int *piv = (int *)(Aug + (int64_t)3 * n * n + 2 * n);
  int bits = 0;
  const int nsq = n * n;
  for (int q0 = lane; q0 < nsq; q0 += UNR * WT) {
    double r[UNR], d2[UNR], asp[UNR], d1[UNR], sv[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      const bool in = q < nsq;
      const int i = q / n, j = q % n;
      r[u] = in ? Aug[(int64_t)i * ld + j] : 0.0;
      d2[u] = in ? ch[j].d2 : 0.0;
      asp[u] = (in && j < no) ? ch[j].asp : 0.0;
      d1[u] = (in && i == j) ? ch[i].d1 : 0.0;
      sv[u] = (in && i == j) ? ch[i].s : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      if (q >= nsq) continue;
      const int i = q / n, j = q % n;
      A32[(int64_t)i * ld32 + j] = (float)(d1[u] - r[u] * d2[u]);
      if (j < no) A32[(int64_t)i * ld32 + n + j] = (float)(r[u] * asp[u] - sv[u]);
    }
  }
  // ||M||_inf from the FP64 entries (row sums of |d1 - R d2|)
  double anrm = 0.0;
  for (int i = lane; i < n; i += WT) {
    double rs = 0.0;
    for (int j = 0; j < n; ++j)
      rs += fabs((i == j ? ch[i].d1 : 0.0) - Aug[(int64_t)i * ld + j] * ch[j].d2);
    anrm = fmax(anrm, rs);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) anrm = fmax(anrm, __shfl_xor(anrm, off));
  wave_sync();
  if (wave_lu_solve(A32, n, ld32, no, W, piv)) bits |= RM_E_SINGULAR;
  // Z in FP64
  const int nz = n * no;
  double zmax = 0.0;
  for (int q = lane; q < nz; q += WT) {
    const int i = q / no, j = q % no;
    const double z = (double)A32[(int64_t)i * ld32 + n + j];
    Aug[(int64_t)i * ld + n + j] = z;
    zmax = fmax(zmax, fabs(z));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) zmax = fmax(zmax, __shfl_xor(zmax, off));
  wave_sync();
  const double tol = 4.0 * sqrt((double)n) * 0x1p-53 * anrm;
  bool conv = false;
  double dprev = 1e300;
  double rmax = wave_residual(Aug, ld, Aug + n, ch, n, no, A32 + n, ld32);
  for (int it = 0; it < L.refine_iters; ++it) {
    if (rmax == 0.0) {
      conv = true;
      break;
    }
    if (!(rmax < 1e300)) break;  // not finite
    wave_lu_resolve(A32, n, ld32, no, piv, W);
    double dmax = 0.0;
    zmax = 0.0;
    for (int q = lane; q < nz; q += WT) {
      const int i = q / no, j = q % no;
      const double dz = (double)A32[(int64_t)i * ld32 + n + j];
      const double z = Aug[(int64_t)i * ld + n + j] + dz;
      Aug[(int64_t)i * ld + n + j] = z;
      zmax = fmax(zmax, fabs(z));
      dmax = fmax(dmax, fabs(dz));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      zmax = fmax(zmax, __shfl_xor(zmax, off));
      dmax = fmax(dmax, __shfl_xor(dmax, off));
    }
    wave_sync();
    // the correction is below the rounding of Z itself
    if (dmax <= 0x1p-50 * zmax) {
      conv = true;
      break;
    }
    rmax = wave_residual(Aug, ld, Aug + n, ch, n, no, A32 + n, ld32);
    // corrections no longer contract: the FP64 floor of this system, if the
    // residual passes the backward-error test there
    if (dmax > 0.5 * dprev) {
      conv = rmax <= tol * zmax;
      break;
    }
    dprev = dmax;
  }
  if (!conv) {
    // as LAPACK's dsgesv does: the FP32 factors cannot refine this system
    // (cond(M) u_32 near 1, e.g. within ~1e-6 Ry of a pole at 200
    // channels), so solve it again with the FP64 factorisation from R,
    // still in Aug's left half
    bits |= RM_E_REFINE_NOCONV;
    for (int q0 = lane; q0 < nsq; q0 += UNR * WT) {
      double r[UNR], d2[UNR], asp[UNR], d1[UNR], sv[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        const bool in = q < nsq;
        const int i = q / n, j = q % n;
        r[u] = in ? Aug[(int64_t)i * ld + j] : 0.0;
        d2[u] = in ? ch[j].d2 : 0.0;
        asp[u] = (in && j < no) ? ch[j].asp : 0.0;
        d1[u] = (in && i == j) ? ch[i].d1 : 0.0;
        sv[u] = (in && i == j) ? ch[i].s : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        if (q >= nsq) continue;
        const int i = q / n, j = q % n;
        Aug[(int64_t)i * ld + j] = d1[u] - r[u] * d2[u];
        if (j < no) Aug[(int64_t)i * ld + n + j] = r[u] * asp[u] - sv[u];
      }
    }
    wave_sync();
    if (wave_lu_solve<double, 1>(Aug, n, ld, no, W)) bits |= RM_E_SINGULAR;
  }
  return bits;
}

// One symmetry at one energy, one wavefront.  Returns RM_E_* bits.
template <bool F32>
__device__ int match_one(const MatchLaunch &L, int s, int e, WaveLds &W) {
  const SymDev &S = L.syms[s];
  const int lane = lane_id();
  const int n = S.n;
  const int ld = 2 * n;
  const double Ee = L.E[e];
  double *Aug = L.work + (int64_t)e * L.work_estride + L.work_off[s];
  double *Kb = Aug + (int64_t)2 * n * n;
  ChanSlot *ch = L.chan + (int64_t)e * L.chan_estride + L.chan_off[s];
  int *rank = (int *)ch;  // reused once the channel slots are consumed
  const int no = count_open(S, Ee);
  if (L.n_open_out && s == 0 && lane == 0) L.n_open_out[e] = no;
  if (no == 0) {
    if (L.K_out && s == 0) {
      double *Ko = L.K_out + (int64_t)e * n * n;
      for (int idx = lane; idx < n * n; idx += WT) Ko[idx] = 0.0;
    }
    return RM_E_NO_OPEN;
  }
  int bits = 0;
  const bool k_given = (L.K_in != nullptr) && s == 0;
  if (!k_given && F32) {
    bits |= wave_channel_functions(S, Ee, ch);
    wave_sync();
    bits |= wave_solve_fp32(L, S, Aug, Kb, ch, no, W);
  } else if (!k_given) {
    // with the asymptotic expansion the propagation kernel has assembled
    // the system at A (and set the channel-function bits)
    if (S.gl_terms == 0) {
      bits |= wave_channel_functions(S, Ee, ch);
      wave_sync();
      // [D1 - R D2 | R[:, P] diag(a s'_P) - diag(s_P)], R already in place
      const int nsq = n * n;
      for (int q0 = lane; q0 < nsq; q0 += UNR * WT) {
        double r[UNR], d2[UNR], asp[UNR], d1[UNR], sv[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int q = q0 + u * WT;
          const bool in = q < nsq;
          const int i = q / n, j = q % n;
          r[u] = in ? Aug[(int64_t)i * ld + j] : 0.0;
          d2[u] = in ? ch[j].d2 : 0.0;
          asp[u] = (in && j < no) ? ch[j].asp : 0.0;
          d1[u] = (in && i == j) ? ch[i].d1 : 0.0;
          sv[u] = (in && i == j) ? ch[i].s : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int q = q0 + u * WT;
          if (q >= nsq) continue;
          const int i = q / n, j = q % n;
          Aug[(int64_t)i * ld + j] = d1[u] - r[u] * d2[u];
          if (j < no) Aug[(int64_t)i * ld + n + j] = r[u] * asp[u] - sv[u];
        }
      }
      wave_sync();
    }
    if (wave_lu_solve(Aug, n, ld, no, W)) bits |= RM_E_SINGULAR;
  }
  if (!k_given) {
    // K = sym(Z[0:no, 0:no]) -> Kb (ld n)
    const int nk = no * no;
    for (int q0 = lane; q0 < nk; q0 += UNR * WT) {
      double a[UNR], b[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        const int i = q / no, j = q % no;
        a[u] = q < nk ? Aug[(int64_t)i * ld + n + j] : 0.0;
        b[u] = q < nk ? Aug[(int64_t)j * ld + n + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        if (q < nk) Kb[(int64_t)(q / no) * n + q % no] = 0.5 * (a[u] + b[u]);
      }
    }
    if (L.sigma) {
      // dipole amplitudes of the K-matrix solutions: with u_ij'(a) =
      // (a s'_j delta_ij + d2_i Z_ij) / a over every channel i (Z = [K; X]),
      // v_j = sum_i u_ij'(a) g_i
      const double *g = Aug + (int64_t)3 * n * n;
      double *v = Aug + (int64_t)3 * n * n + n;
      for (int j0 = 0; j0 < no; j0 += WT) {
        const int j = j0 + lane;
        double acc = 0.0;
        for (int i0 = 0; i0 < n; i0 += UNR) {
          double z[UNR], h[UNR];
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            const int i = i0 + u;
            z[u] = (i < n && j < no) ? Aug[(int64_t)i * ld + n + j] : 0.0;
            h[u] = i < n ? ch[i].d2 * g[i] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < UNR; ++u) acc = fma(h[u], z[u], acc);
        }
        if (j < no) v[j] = (ch[j].asp * g[j] + acc) / S.a;
      }
    }
  }
  // rank of each open channel among the open channels' input indices
  if (L.K_out || k_given) {
    wave_sync();
    for (int i = lane; i < no; i += WT) {
      const int pi = S.perm[i];
      int r = 0;
#pragma unroll 8
      for (int j = 0; j < no; ++j) r += (S.perm[j] < pi);
      rank[i] = r;
    }
  }
  wave_sync();
  if (k_given) {
    const double *Ki = L.K_in + (int64_t)e * n * n;  // input order, ld n
    const int nk = no * no;
    for (int q0 = lane; q0 < nk; q0 += UNR * WT) {
      double v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        v[u] = q < nk ? Ki[(int64_t)rank[q / no] * n + rank[q % no]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        if (q < nk) Kb[(int64_t)(q / no) * n + q % no] = v[u];
      }
    }
    wave_sync();
  }
  int nonfinite = 0;
  if (L.K_out && s == 0) {
    double *Ko = L.K_out + (int64_t)e * n * n;
    for (int idx = lane; idx < n * n; idx += WT) {
      const int r = idx / n, c = idx % n;
      if (r >= no || c >= no) Ko[idx] = 0.0;
    }
    const int nk = no * no;
    for (int q0 = lane; q0 < nk; q0 += UNR * WT) {
      double v[UNR];
      int ri[UNR], rj[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = q0 + u * WT;
        const bool in = q < nk;
        v[u] = in ? Kb[(int64_t)(q / no) * n + q % no] : 0.0;
        ri[u] = in ? rank[q / no] : 0;
        rj[u] = in ? rank[q % no] : 0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        if (q0 + u * WT >= nk) continue;
        if (!isfinite(v[u])) nonfinite = 1;
        Ko[(int64_t)ri[u] * n + rj[u]] = v[u];
      }
    }
  }
  if (L.do_t) {
    // Y in Aug's columns [no, 2 no); A in [0, no) and V in K's place, or
    // Q in K's place and V in [0, no)
    double *pv = (L.sigma && !k_given) ? Aug + (int64_t)3 * n * n + n : nullptr;
    wave_sync();
    int route = T_ROUTE_A;
    if (wave_tstep(Aug, ld, Kb, n, no, W, L.omega != nullptr, pv, L, e, route))
      bits |= RM_E_SINGULAR;
    if (L.omega)
      nonfinite |= route == T_ROUTE_A
                       ? wave_omega(S, L.n_target_out, Aug + no, ld, Aug, ld,
                                    true, Kb, n, no,
                                    L.omega + (int64_t)e * L.omega_stride)
                       : wave_omega(S, L.n_target_out, Aug + no, ld, Kb, n,
                                    false, Aug, ld, no,
                                    L.omega + (int64_t)e * L.omega_stride);
    if (pv) {
      // sigma += (4 pi^2 alpha a0^2 / 3) omega (1/pi) |L^-1 v|^2
      double s2 = 0.0;
      for (int j = lane; j < no; j += WT) s2 = fma(pv[j], pv[j], s2);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) s2 += __shfl_xor(s2, o);
      const double c = 4.0 * M_PI * 7.2973525693e-3 * 28.00285205 / 3.0;
      const double add = c * (Ee - L.e0) * s2;
      if (!isfinite(add)) nonfinite = 1;
      if (lane == 0) L.sigma[e] += add;
    }
  }
  if (nonfinite) bits |= RM_E_NONFINITE;
  wave_sync();
  return wave_or(bits);
}

// Radiation-damped photoionization, one symmetry at one energy.  With the
// pole energies E_k - i Gamma_k/2 the pole sums are complex, R_c = R_re +
// i R_im and g_c = g_re + i g_im (the pole-sum kernels' parts 1 and 2), and
// the driven solution of (E - H_eff) psi = D Psi_0 with outgoing waves
// outside satisfies
//     (diag(d1) - R_c diag(d2)) x = -g_c,
// d1 = c + i s, d2 = a (c' + i s') on open channels (u = (c + i s) alpha)
// and the closed function (e, a e') on closed ones; its flux into the open
// channels is sum_f |alpha_f|^2 (c s' - s c' = 1), and sigma +=
// (4 pi alpha a0^2 / 3) omega sum_f |alpha_f|^2.  The complex system is
// solved as the real 2n x 2n system [[A_r, -A_i], [A_i, A_r]] [x_r; x_i] =
// [-g_re; -g_im] by the wavefront LU.  Returns RM_E_* bits.
__device__ int match_one_damped(const MatchLaunch &L, int s, int e,
                                WaveLds &W) {
  const SymDev &S = L.syms[s];
  const int lane = lane_id();
  const int n = S.n, n2 = 2 * n, ld = 2 * n + 2;
  const double Ee = L.E[e];
  double *Sys = L.work + (int64_t)e * L.work_estride + L.work_off[s];
  const double *Rre = Sys + (int64_t)n2 * ld;
  const double *Rim = Rre + (int64_t)n * n;
  const double *gre = Rim + (int64_t)n * n;
  const double *gim = gre + n;
  ChanSlot *ch = L.chan + (int64_t)e * L.chan_estride + L.chan_off[s];
  const int no = count_open(S, Ee);
  if (no == 0) return RM_E_NO_OPEN;
  int bits = wave_channel_functions(S, Ee, ch);
  wave_sync();
  const int nsq = n * n;
  for (int q0 = lane; q0 < nsq; q0 += UNR * WT) {
    double rr[UNR], ri[UNR], d2[UNR], asp[UNR], d1[UNR], sv[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      const bool in = q < nsq;
      const int i = q / n, j = q % n;
      rr[u] = in ? Rre[q] : 0.0;
      ri[u] = in ? Rim[q] : 0.0;
      d2[u] = in ? ch[j].d2 : 0.0;
      asp[u] = in ? ch[j].asp : 0.0;
      d1[u] = (in && i == j) ? ch[i].d1 : 0.0;
      sv[u] = (in && i == j) ? ch[i].s : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = q0 + u * WT;
      if (q >= nsq) continue;
      const int i = q / n, j = q % n;
      const double ar = d1[u] - (rr[u] * d2[u] - ri[u] * asp[u]);
      const double ai = sv[u] - (rr[u] * asp[u] + ri[u] * d2[u]);
      Sys[(int64_t)i * ld + j] = ar;
      Sys[(int64_t)i * ld + n + j] = -ai;
      Sys[(int64_t)(n + i) * ld + j] = ai;
      Sys[(int64_t)(n + i) * ld + n + j] = ar;
    }
  }
  for (int i = lane; i < n; i += WT) {
    Sys[(int64_t)i * ld + n2] = -gre[i];
    Sys[(int64_t)(n + i) * ld + n2] = -gim[i];
  }
  wave_sync();
  if (wave_lu_solve<double, 2>(Sys, n2, ld, 1, W)) bits |= RM_E_SINGULAR;
  double s2 = 0.0;
  for (int f = lane; f < no; f += WT) {
    const double xr = Sys[(int64_t)f * ld + n2];
    const double xi = Sys[(int64_t)(n + f) * ld + n2];
    s2 = fma(xr, xr, fma(xi, xi, s2));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s2 += __shfl_xor(s2, o);
  const double c = 4.0 * M_PI * 7.2973525693e-3 * 28.00285205 / 3.0;
  const double add = c * (Ee - L.e0) * s2;
  if (!isfinite(add)) bits |= RM_E_NONFINITE;
  if (lane == 0) L.sigma[e] += add;
  wave_sync();
  return wave_or(bits);
}

#ifndef RM_MATCH_DEVICE_ONLY
// MODE 0: FP64 solve; 1: FP32 solve refined in FP64; 2: damped
// photoionization; 3: FP64 solve for symmetries of more than 600 channels.
// Separate instantiations keep each kernel's registers its own.  MODE 0
// runs two wavefronts per SIMD (256 registers each, some spilled): its
// serial phases (panels, diagonal blocks) wait on memory round trips that
// the second wavefront covers, 4 % faster at 200 channels than one
// wavefront per SIMD with every register; at 1815 channels the spills of
// the larger panels cost more than that (10 % slower), so MODE 3 is the
// same code at one wavefront per SIMD.
template <int MODE>
__global__ __launch_bounds__(WT *WPB)
__attribute__((amdgpu_waves_per_eu(MODE == 0 ? 2 : 1, MODE == 0 ? 2 : 1)))
void match_kernel(MatchLaunch L) {
  __shared__ WaveLds lds[WPB];
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int gw = blockIdx.x * WPB + wv;  // global wave id
  int e = gw;
  for (;;) {
    if (L.counter) {
      int v = 0;
      if (lane == 0) v = atomicAdd(L.counter, 1);
      e = __builtin_amdgcn_readfirstlane(v);  // wavefront-uniform
    }
    if (e >= L.m) break;
    int stat = 0;
    for (int s = 0; s < L.n_sym; ++s) {
      if constexpr (MODE == 2)
        stat |= match_one_damped(L, s, e, lds[wv]);
      else
        stat |= match_one<MODE == 1>(L, s, e, lds[wv]);
    }
    if (lane == 0 && L.status && stat) atomicOr(&L.status[e], stat);
    if (!L.counter) break;
  }
}

hipError_t launch_match(const MatchLaunch &L, hipStream_t st) {
  if (L.m <= 0) return hipSuccess;
  const int waves = L.counter ? std::max(1, std::min(L.grid * WPB, L.m)) : L.m;
  const unsigned blocks = (unsigned)((waves + WPB - 1) / WPB);
  if (L.damped)
    hipLaunchKernelGGL(match_kernel<2>, dim3(blocks), dim3(WT * WPB), 0, st, L);
  else if (L.solve_fp32)
    hipLaunchKernelGGL(match_kernel<1>, dim3(blocks), dim3(WT * WPB), 0, st, L);
  else if (L.n_max > 600)
    hipLaunchKernelGGL(match_kernel<3>, dim3(blocks), dim3(WT * WPB), 0, st, L);
  else
    hipLaunchKernelGGL(match_kernel<0>, dim3(blocks), dim3(WT * WPB), 0, st, L);
  return hipGetLastError();
}

#endif  // RM_MATCH_DEVICE_ONLY

}  // namespace rmx
