// Internal declarations shared by the HIP translation units of librmatrix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rmatrix.h"

namespace rmx {

// Padding granularity of channels and poles in the staged W layouts.
constexpr int kChanPad = 32;
constexpr int kPolePad = 64;
constexpr double kPadPole = 1.0e30;  // padding poles sit far from any energy

// A symmetry resident on one device.  Channels are stored sorted by
// threshold (stable), so at any energy the open channels are a prefix.
struct Sym {
  int device;
  int n, nh;            // channels, poles
  int n_pad, nh_pad;    // padded to kChanPad / kPolePad
  double a, z, g;
  int n_target;         // max target level + 1
  // device arrays
  double *E_pole;       // [nh_pad] ascending, padding = kPadPole
  double *Wt;           // [nh_pad][n_pad] FP64, k-major, zero padded
  float *W32c;          // [n_pad][nh_pad] FP32, channel-major
  uint16_t *Whc, *Wlc;  // [n_pad][nh_pad] BF16 split, channel-major:
                        // w = hi + lo + O(2^-16 |w|)
  double *e_thr;        // [n] sorted
  int32_t *l;           // [n] (sorted order)
  int32_t *perm;        // [n] sorted position -> input channel
  int32_t *inv;         // [n] input channel -> sorted position
  int32_t *tptr;        // [n_target+1] CSR: channels (sorted positions) per
  int32_t *tch;         // [n]           target level, ascending
  // host copies
  double *h_e_thr;      // [n] sorted
  int32_t *h_perm;
};

// Per-energy channel data written by the channel-function kernel, sorted
// channel order: (d1, d2, s, a s') with d1 = c, d2 = a c' for open channels
// and (e, a e') of the closed-channel function for closed ones.
struct ChanSlot {
  double d1, d2, s, asp;
};

// ---- launchers (return hipError_t of the launch) ----

hipError_t launch_chanfn(const Sym &s, const double *E, int64_t m,
                         ChanSlot *chan, int32_t *n_open, int32_t *status,
                         hipStream_t st);

// Pole sum (Sec. 6, Eq. 1-2), FP64 MFMA over all poles.  Writes
// R[e][i][j] (sorted channel order) at R + e*r_estride + i*r_ld + j,
// scaled by 1/(2a), both triangles.
hipError_t launch_polesum_f64(const Sym &s, const double *E, int64_t m,
                              double *R, int64_t r_estride, int r_ld,
                              hipStream_t st);

// Mixed-precision pole sum: far poles in FP32 or split-BF16 MFMA with FP32
// accumulation, then the FP64 near-pole correction for |E_k - E| < delta.
hipError_t launch_polesum_mixed(const Sym &s, int prec, double delta,
                                const double *E, int64_t m, double *R,
                                int64_t r_estride, int r_ld, hipStream_t st);

// Matching -> K -> T -> Omega for m energies.  work: per energy a block of
// 3 n^2 doubles whose first 2 n^2 (row-major, ld 2n) hold R on entry in the
// left half (sorted order).  K_out (may be null): [m][n][n] open-open block
// in input-channel order.  omega (may be null): accumulated.
struct MatchArgs {
  const ChanSlot *chan;
  const int32_t *n_open;
  double *work;
  int64_t work_stride;  // doubles per energy
  int m;
  double *K_out;        // nullable
  double *omega;        // nullable
  int64_t omega_stride;
  int n_target_out;     // Omega row has n_target_out*(n_target_out+1)/2
  int32_t *status;      // nullable
  int do_t;             // 1: compute T and Omega
  int solve_fp32;
  int refine_iters;
};
hipError_t launch_match(const Sym &s, const MatchArgs &a, hipStream_t st);

// Omega from given K (rm_collision_strengths).
hipError_t launch_t_omega_from_k(const Sym &s, const double *K,
                                 const int32_t *n_open, int64_t m,
                                 double *work, int64_t work_stride,
                                 double *omega, int n_target_out,
                                 hipStream_t st);

hipError_t launch_fill(double *p, int64_t count, double v, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t v,
                           hipStream_t st);
// Copy R from sorted to input order into a dense [m][n][n] array.
hipError_t launch_unsort_square(const Sym &s, const double *src,
                                int64_t src_estride, int src_ld, double *dst,
                                int64_t m, hipStream_t st);
hipError_t launch_unsort_chan(const Sym &s, const ChanSlot *chan, int64_t m,
                              double *out, hipStream_t st);

}  // namespace rmx
