// Internal declarations shared by the HIP translation units of librmatrix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "../../include/rmatrix.h"

namespace rmx {

// Padding granularity of channels and poles in the staged W layouts.
constexpr int kChanPad = 32;
constexpr int kPolePad = 64;
constexpr double kPadPole = 1.0e30;  // padding poles sit far from any energy
// The T step's well-conditioned route (the real 2n x 2n form of
// (1 - iK) W = 1 with its right-hand sides, 6 n^2 doubles) runs at few
// energies, so its buffers form a small pool of slots that a wavefront
// takes by compare-and-swap on a flag and gives back when done; with every
// slot taken the energy takes the route through Z = L^-1 K instead (no
// wavefront ever waits).
constexpr int kMatchWpb = 4;     // wavefronts per matching workgroup
constexpr int kTExtSlots = 64;   // pool slots of an allocating sweep
constexpr int kTExtSlotsArena = 16;  // of a sweep that may not allocate
__host__ __device__ inline int64_t t_ext_doubles(int n) {
  return (int64_t)6 * n * n;
}

// The asymptotic expansion beyond A works on blocks of kGlCols open
// channels; its per-energy scratch (after the symmetry's workspace) holds a
// doubled ring of 2 Q coefficient slots (Q = max(lmax, 2) + 1), two slots
// of the coupling products, the sums g and g', and two slots for the final
// product with R, each slot n rows of 2 kGlCols doubles (real | imaginary).
// Doubles of one energy's matching workspace of an n-channel symmetry:
// [M | B] n x 2n, K n x n, 2n for photoionization, n pivots.
__host__ __device__ inline int64_t match_work_doubles(int n) {
  return (int64_t)3 * n * n + 3 * n;
}

constexpr int kGlCols = 16;
constexpr int kGlMaxTerms = 200;
__host__ __device__ inline int gl_ring(int lmax) { return (lmax > 2 ? lmax : 2) + 1; }
__host__ __device__ inline int64_t gl_doubles(int n, int lmax) {
  return (int64_t)(2 * gl_ring(lmax) + 6) * n * 2 * kGlCols;
}

// Device-side view of one symmetry (plain data, copied into a descriptor
// table that the grouped kernels index by symmetry number).
struct SymDev {
  int n, nh, n_pad, nh_pad;
  int n_target;
  double a, z, g;
  const double *E_pole;       // [nh_pad] ascending, padding = kPadPole
  const double *Wt;           // [nh_pad][n_pad] FP64, pole-major
  const float *W32c;          // [n_pad][nh_pad] FP32, channel-major
  const uint16_t *Whc, *Wlc;  // [n_pad][nh_pad] BF16 split, channel-major
  const double *e_thr;        // [n] sorted
  const int32_t *l;           // [n] sorted order
  const int32_t *perm;        // [n] sorted position -> input channel
  const int32_t *tgt;         // [n] sorted position -> target level
  int ntu;                    // target levels that hold a channel
  const int32_t *ut;          // [ntu] those levels, ascending
  const double *G;            // [n][ntu] 0/1, channel -> used level
  const double *GT;           // [ntu][n] its transpose
  int np, np_pad;             // pairs i <= j (row-major upper triangle)
  const int32_t *pair_ij;     // [np_pad] (i << 16) | j
  const uint16_t *Ph, *Pl;    // [np_pad][nh_pad] BF16 hi/lo of w_ik w_jk
  const float *P32;           // [np_pad][nh_pad] FP32 w_ik w_jk
  const double *P64;          // [np_pad][nh_pad] FP64 w_ik w_jk
  const double *dip;          // [nh_pad] bound-free dipoles, or null
  const double *gam;          // [nh_pad] radiative widths Gamma_k, or null
  // outer-region propagation from a to A (n_sec = 0: none): sector s
  // rotates the reduced R-matrix by O_s (X <- O_s^T X O_s) and then steps
  // it across width h_sec with eigenvalues eps_s; O_{n_sec} returns to the
  // channel basis.  Sorted channel order, leading dimension n.
  int n_sec;
  double A, h_sec;
  double r_match;             // radius of the matching: A with sectors, else a
  const double *prop_O;       // [n_sec + 1][n][n]
  const double *prop_eps;     // [n_sec][n]
  // asymptotic expansion at A (gl_terms = 0: matching to Coulomb functions):
  // gl_beta [n][lmax n], row i holds beta^lam_im / A^lam for lam = 1..lmax
  int gl_terms, lmax;
  const double *gl_beta;
};

// A symmetry resident on one device.  Channels are stored sorted by
// threshold (stable), so at any energy the open channels are a prefix.
struct Sym {
  int device;
  int n, nh;            // channels, poles
  int n_pad, nh_pad;    // padded to kChanPad / kPolePad
  double a, z, g;
  int n_target;         // max target level + 1
  // device arrays (owned)
  double *E_pole;
  double *Wt;
  float *W32c;
  uint16_t *Whc, *Wlc;  // w = hi + lo + O(2^-16 |w|)
  double *e_thr;
  int32_t *l;
  int32_t *perm;
  int32_t *inv;         // [n] input channel -> sorted position
  int32_t *tgt;
  int ntu;
  int32_t *ut;
  double *G, *GT;
  int np, np_pad;       // channel pairs, padded to the pair-block size
  int32_t *pair_ij;
  uint16_t *Ph, *Pl;    // pair products, formed on first use (owned)
  float *P32;
  double *P64;
  double *dip = nullptr;  // [nh_pad] dipoles with the initial state (owned)
  double *gam = nullptr;  // [nh_pad] radiative widths of the poles (owned)
  int n_sec = 0;          // outer-region sectors (0: match at r = a)
  double A = 0.0, h_sec = 0.0;
  double *prop_O = nullptr, *prop_eps = nullptr;  // owned
  int lmax = 0, gl_terms = 0;   // multipole order; expansion terms (0: off)
  double *gl_beta = nullptr;    // [n][lmax n] beta / A^lam, sorted (owned)
  // host copies
  double *h_e_thr;      // [n] sorted
  int32_t *h_perm;
  SymDev dev() const {
    SymDev d;
    d.n = n; d.nh = nh; d.n_pad = n_pad; d.nh_pad = nh_pad;
    d.n_target = n_target; d.a = a; d.z = z; d.g = g;
    d.E_pole = E_pole; d.Wt = Wt; d.W32c = W32c; d.Whc = Whc; d.Wlc = Wlc;
    d.e_thr = e_thr; d.l = l; d.perm = perm; d.tgt = tgt;
    d.ntu = ntu; d.ut = ut; d.G = G; d.GT = GT;
    d.np = np; d.np_pad = np_pad; d.pair_ij = pair_ij;
    d.Ph = Ph; d.Pl = Pl; d.P32 = P32; d.P64 = P64; d.dip = dip; d.gam = gam;
    d.n_sec = n_sec; d.A = A; d.h_sec = h_sec;
    d.r_match = n_sec > 0 ? A : a;
    d.prop_O = prop_O; d.prop_eps = prop_eps;
    d.gl_terms = n_sec > 0 ? gl_terms : 0;
    d.lmax = lmax;
    d.gl_beta = gl_beta;
    return d;
  }
};

// Per-energy channel data, sorted channel order: (d1, d2, s, a s') with
// d1 = c, d2 = a c' for open channels and (e, a e') of the closed-channel
// function for closed ones.
struct ChanSlot {
  double d1, d2, s, asp;
};

// Work item of the grouped pole-sum kernels: symmetry, two tile
// coordinates (meaning per kernel) and an energy group.
struct PsItem {
  int sym, x, y, grp;
};

// Where the pole sum writes R of symmetry s at chunk energy e:
// out + e*estride + off[s] + i*(ld_mult*n_s) + j.
struct PsOut {
  double *out;
  int64_t estride;
  const int64_t *off;   // device [n_sym]
  int ld_mult;
};

// Tile variants of the pole-sum kernels (chosen by the autotuner).
enum PsVariant {
  PS_F64_T32_E16 = 0,   // FP64, 32x32 tile pairs, 16 energies per WG
  PS_MX_J16_E8 = 1,     // mixed, 16 column blocks, 8 energies per WG
  PS_MX_J8_E8 = 2,      // mixed, 8 column blocks, 8 energies per WG
  PS_MX_J16_E4 = 3,     // mixed, 16 column blocks, 4 energies per WG
  PS_PD = 4,            // mixed, pair-major GEMM over precomputed w_ik w_jk
  PS_PD64 = 5           // FP64, pair-major GEMM
};
constexpr int kPairBlock = 256;   // pairs per pair-major workgroup tile

// ---- launchers (return the hipError_t of the launch) ----

hipError_t launch_chanfn(const Sym &s, const double *E, int64_t m,
                         ChanSlot *chan, int32_t *n_open, int32_t *status,
                         hipStream_t st);

// Grouped pole sum (Sec. 6, Eq. 1-2) over a table of work items that may
// span several symmetries.  FP64 variants use MFMA over every pole; mixed
// variants use FP32 or split-BF16 MFMA over the far poles, |E_k - E| >=
// band, and add the near tier (|E_k - E| < delta, FP64 operands) and the
// band tier (FP32 operands, FP64 products and sum) in their epilogues.  With a counter (device int
// holding 0) the grid is persistent and pulls items from it.
struct PsLaunch {
  const SymDev *syms;
  const PsItem *items;
  int n_items;
  int *counter;         // nullable
  int grid;             // persistent grid size (used with counter)
  const double *E;
  int m;
  PsOut out;
  int prec;
  double delta;         // near tier: FP64 operands
  double band;          // band tier (>= delta): FP32 operands, FP64 sum
  // FP64 scaled-W variant only: 0 the weights 1/(E_k - E); 1 and 2 the
  // real and imaginary parts of 1/(E_k - i Gamma_k/2 - E) (damped poles)
  int part;
};
hipError_t launch_polesum(const PsLaunch &L, int variant, hipStream_t st);
hipError_t launch_polesum_pd(const PsLaunch &L, hipStream_t st);
hipError_t launch_polesum_pd64(const PsLaunch &L, hipStream_t st);
hipError_t launch_pd64_build(const Sym &s, hipStream_t st);
// Form the pair products of s for prec (FP32 or BF16X3) into its planes.
hipError_t launch_pd_build(const Sym &s, int prec, hipStream_t st);
int ps_energy_group(int variant);         // energies per work item
// Tile items of one symmetry for a variant: (x, y) pairs, in order.
void ps_tiles(const Sym &s, int variant, std::vector<std::pair<int, int>> &out);

// Channel functions, matching, K, T and Omega: one wavefront per energy,
// looping over every symmetry (so it owns that energy's Omega row).  With a
// counter the grid is persistent.
struct MatchLaunch {
  const SymDev *syms;
  int n_sym;
  const double *E;
  int m;
  // photoionization: the dipole pole sum g of each symmetry sits after its
  // K block in the workspace ([Aug 2n^2 | K n^2 | g n | v n]); sigma[e] is
  // accumulated over the symmetries (nullable)
  double *sigma;
  double e0;
  double *work;               // [M | B] (n x 2n), K (n x n), 2n, n pivots
  int64_t work_estride;
  const int64_t *work_off;    // device [n_sym]
  ChanSlot *chan;
  int64_t chan_estride;
  const int64_t *chan_off;    // device [n_sym]
  int32_t *n_open_out;        // nullable, symmetry 0 only
  double *K_out;              // nullable, symmetry 0 only: [m][n][n]
  const double *K_in;         // nullable, symmetry 0 only (skip matching)
  double *omega;              // nullable
  int64_t omega_stride;
  int n_target_out;
  int32_t *status;            // nullable
  int do_t;
  int *counter;               // nullable
  int grid;
  int solve_fp32;             // FP32 factorisation refined in FP64
  int refine_iters;           // at most this many corrections
  // radiation-damped photoionization: per symmetry the workspace holds the
  // 2n x 2n real form of the complex driven system (leading dimension
  // 2n + 2), then R_re, R_im (n x n each) and g_re, g_im (n each)
  int damped;
  // the T step's complex-system pool (nullable): ext_slots slots of
  // ext_estride doubles (at least t_ext_doubles(n) of every symmetry) at
  // ext + slot * ext_estride, slot q free while ext_flags[q] == 0 (the
  // flags start at zero)
  double *ext;
  int64_t ext_estride;
  int *ext_flags;
  int ext_slots;
  int n_max;                  // the largest symmetry's channels (kernel choice)
};
hipError_t launch_match(const MatchLaunch &L, hipStream_t st);
// R(a) -> R(A) for the symmetries with outer-region sectors (same launch
// description as the matching; run between the pole sum and the matching).
hipError_t launch_propagate(const MatchLaunch &L, hipStream_t st);

// Dipole pole sum g_i(E) = (1/sqrt2) sum_k w_ik d_k / (E_k - E) of one
// symmetry (sorted channel order) at the m energies E, written to
// out + e*estride + off + i.
// part as for PsLaunch: 0 undamped, 1 and 2 the real and imaginary parts
// with damped pole energies E_k - i Gamma_k/2.
hipError_t launch_dip_polesum(const SymDev &S, const double *E, int m,
                              double *out, int64_t estride, int64_t off,
                              hipStream_t st, int part = 0);

hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v,
                           hipStream_t st);
// Copy R from sorted to input order into a dense [m][n][n] array.
hipError_t launch_unsort_square(const Sym &s, const double *src,
                                int64_t src_estride, int src_ld, double *dst,
                                int64_t m, hipStream_t st);

// rm_profile stage timing: while rm_profile(1) is in force, the launches a
// scope issues on `st` are bracketed by events recorded under `stage`.
struct ProfileScope {
  ProfileScope(int stage, hipStream_t st);
  ~ProfileScope();
  hipEvent_t end_ = nullptr;
  hipStream_t st_;
};

}  // namespace rmx
