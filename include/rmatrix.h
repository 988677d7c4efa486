/*
 * rmatrix.h -- C ABI of the MI355X (gfx950) R-matrix outer-region sweep.
 *
 * The library evaluates, for every energy E of a mesh and every symmetry
 * (LS-pi or J-pi partial wave) of a scattering system, the chain that the
 * outer-region module of the parallel Breit-Pauli / DARC R-matrix codes runs
 * (McLaughlin & Ballance, "Petascale computations for large-scale atomic and
 * molecular collisions", Sec. 3 and Sec. 6):
 *
 *   R_ij(E) = (1/2a) sum_k w_ik w_jk / (E_k - E)        Sec. 6, Eq. 1-2
 *   match R(E) at r = a to Coulomb functions F_l, G_l (open channels) and
 *   decaying Whittaker functions (closed channels)  ->  K-matrix (open-open)
 *   T = 2iK (1 - iK)^-1
 *   Omega(t, t') += (g/2) sum_{i in t, j in t', open} |T_ij|^2
 *
 * Eq. 1 is printed as sum_k W_ik W_kj / (E - E_k) with no prefactor; the
 * library uses the Bloch-operator normalisation above (Rydberg energies,
 * Bohr radii, Bloch constant b = 0), which is -1/(2a) times the printed form.
 *
 * Units: energies in Rydberg, radii in Bohr.  All functions are host
 * functions; device pointers must address memory of the current HIP device,
 * and `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 * on `stream` and the call returns without synchronising, except where
 * stated.  No function throws; each returns an rm_status code and, when it is
 * not RM_OK, rm_last_error() describes the failure (thread-local).
 *
 * Argument validation happens before anything is enqueued: an RM_ERR_ARG
 * return has touched no device memory.
 */
#ifndef RMATRIX_H
#define RMATRIX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
enum rm_status {
  RM_OK = 0,
  RM_ERR_ARG = 1,      /* invalid argument; nothing enqueued                */
  RM_ERR_NOMEM = 2,    /* device allocation failed                          */
  RM_ERR_HIP = 3,      /* a HIP runtime call failed                         */
  RM_ERR_NUMERIC = 4,  /* iteration did not converge (rm_inner_region);
                          per-energy trouble goes to status[] instead      */
  RM_ERR_STATE = 5     /* handle used on the wrong device or after rm_free  */
};

/* Arithmetic of the pole sum (Sec. 6, Eq. 1-2).  The mixed precisions split
 * the poles of each energy into three tiers by their distance to E:
 *   near  |E_k - E| <  near_delta:  FP64 operands, FP64 sum;
 *   band  near_delta <= |E_k - E| < band_delta:  operands w_ik, w_jk and
 *         d_k rounded to FP32, products and sum in FP64 (the rounding of
 *         each term is then that of a slightly moved pole with slightly
 *         changed amplitudes, not an independent error per matrix entry);
 *   far   the rest: the MFMA precision below with FP32 accumulation.
 * The matching solve is FP64 unless rm_opts.solve_fp32 is set: then the
 * system (D1 - R D2)[K; X] = R[:, P] diag(a s'_P) - [diag(s_P); 0] of each
 * energy is rounded to FP32, LU-factored with partial pivoting and solved in
 * FP32, and the solution refined in FP64 (residual from R in FP64, each
 * correction solved with the FP32 factors) until a correction is below
 * 2^-50 max|[K; X]|, or the corrections stop contracting at a residual with
 * max|r| <= 4 sqrt(n) 2^-53 ||D1 - R D2||_inf max|[K; X]| (the backward-
 * error test of LAPACK's dsgesv), within refine_iters corrections;
 * otherwise (cond u_32 near 1: at 200 channels, energies within about 1e-6
 * Ry of a pole) that energy gets RM_E_REFINE_NOCONV and is solved again
 * with the FP64 factorisation, as dsgesv falls back.  The T step stays
 * FP64. */
enum rm_precision {
  RM_PREC_FP64 = 0,    /* FP64 MFMA over every pole                          */
  RM_PREC_FP32 = 1,    /* FP32 MFMA, FP32 accumulation, far poles only       */
  RM_PREC_BF16X3 = 2   /* split-BF16 (hi*hi + hi*lo + lo*hi) MFMA, FP32
                          accumulation, far poles only                        */
};

/* Per-energy status bits (status[] of rm_sweep_energies / rm_kmatrix).
 * A flagged energy still gets a value; NO_OPEN energies get Omega = 0. */
#define RM_E_NO_OPEN        0x01  /* no channel open: K is 0x0, Omega = 0   */
#define RM_E_SINGULAR       0x02  /* zero pivot in the matching solve       */
#define RM_E_CF_NOCONV      0x04  /* a channel-function iteration hit its cap*/
#define RM_E_NONFINITE      0x08  /* non-finite value in K or T             */
#define RM_E_ON_THRESHOLD   0x10  /* E equals a channel threshold exactly   */
#define RM_E_REFINE_NOCONV  0x20  /* FP32 solve: refinement did not reach
                                     the FP64 test; the energy was solved
                                     again in FP64 (below)                 */
#define RM_E_ASYM_NOCONV    0x40  /* asymptotic expansion at A: a channel's
                                     first omitted term exceeds 1e-6
                                     (rm_set_gailitis)                     */

typedef struct rm_sym *rm_sym_t;  /* one symmetry, device-resident, opaque */

/* One symmetry as the inner region hands it over (all host pointers).
 *   E_pole  [n_poles]          poles E_k, strictly ascending, finite
 *   w       [n_chan*n_poles]   surface amplitudes, row-major: w[i*n_poles+k]
 *   a       boundary radius (> 0)
 *   e_thr   [n_chan]           channel thresholds e_i (finite)
 *   l       [n_chan]           orbital angular momenta, 0 <= l <= 12
 *   target  [n_chan] or NULL   target level of each channel (>= 0); NULL maps
 *                              channel i to level i
 *   z       residual charge seen by the scattered electron (>= 0)
 *   g       statistical weight of the symmetry, e.g. 2J+1 (> 0)
 * Validity domain of the channel functions: z >= 0 and 2 z a > l(l+1) for
 * every channel (r = a lies beyond the centrifugal turning point at all
 * energies); z = 0 requires l = 0 channels or energies with k a > sqrt(l(l+1)).
 */
typedef struct {
  int32_t n_chan;
  int32_t n_poles;
  const double *E_pole;
  const double *w;
  double a;
  const double *e_thr;
  const int32_t *l;
  const int32_t *target;
  double z;
  double g;
} rm_poles_desc;

/* Options; a zero-initialised struct selects the defaults. */
typedef struct {
  int32_t prec;          /* rm_precision                                   */
  double near_delta;     /* Ry, mixed precisions only; 0 -> 1e-3           */
  int32_t solve_fp32;    /* 0: the matching solve in FP64; 1: factored in
                            FP32 and refined in FP64 (below)               */
  int32_t refine_iters;  /* FP32 solve: at most this many FP64 corrections
                            (0 -> 8, at most 100)                          */
  int32_t chunk;         /* energies per internal chunk; 0 -> automatic    */
  uint32_t flags;        /* RM_FLAG_* bits                                 */
  double band_delta;     /* Ry, mixed precisions only: the outer edge of the
                            FP32-operand band; 0 -> 10 near_delta; must be
                            >= near_delta                                  */
} rm_opts;

/* rm_opts.flags: time the pole-sum tile variants on the first plan of each
 * (channels, poles, precision) and keep the fastest (in memory, and in the
 * file named by the environment variable RM_TUNE_CACHE when set). */
#define RM_FLAG_AUTOTUNE 0x1u
/* rm_opts.flags: the pole sum has two forms.  The scaled-W kernels
 * contract (W diag(d)) W^T per energy tile and need nothing beyond W.  The
 * pair form precomputes the products w_ik w_jk (i <= j) once per symmetry
 * and precision, in device memory (8 bytes per pair and pole in FP64, 4 in
 * FP32 or split BF16: 1.3 / 0.66 GB at 200 channels and 8000 poles; not
 * formed above 8 GB, a quarter of free memory, or 32 GB over all live
 * symmetries), and runs one GEMM over them.  Mixed precisions use the pair
 * form where it fits, FP64 uses the scaled-W kernels (with
 * RM_FLAG_AUTOTUNE, whichever times faster).  NO_PAIR_PRODUCTS forces the
 * scaled-W kernels; PAIR_PRODUCTS forces the pair form where it fits.  The
 * two may not be combined (RM_ERR_ARG). */
#define RM_FLAG_NO_PAIR_PRODUCTS 0x2u
#define RM_FLAG_PAIR_PRODUCTS 0x4u
/* rm_opts.flags, rm_photoionization only: radiation damping (below); every
 * other entry point returns RM_ERR_ARG for it. */
#define RM_FLAG_RADIATION_DAMPING 0x8u

/* Load one symmetry (Sec. 3: the poles and amplitudes produced by the
 * inner-region diagonalisation; Sec. 6 Eq. 2: W is the shared operand of
 * every energy's product).  Copies every input to the current device
 * (caller may free its arrays when the call returns; the call synchronises
 * `stream`), sorts channels by threshold internally and stages W in the
 * layouts the kernels read (FP64, FP32 and split BF16).
 * Errors: RM_ERR_ARG (n_chan < 1, n_poles < 1, a <= 0, z < 0, g <= 0,
 * non-ascending or non-finite poles, non-finite amplitudes or thresholds,
 * l outside [0, 12], negative target), RM_ERR_NOMEM, RM_ERR_HIP. */
int rm_load_poles(const rm_poles_desc *desc, rm_sym_t *out, void *stream);

/* Release a handle (synchronises the device first).  NULL is accepted. */
int rm_free(rm_sym_t sym);

/* Channel count, pole count and number of target levels of a handle. */
int rm_sym_info(rm_sym_t sym, int32_t *n_chan, int32_t *n_poles,
                int32_t *n_target);

/* The fused sweep (Sec. 6: the outer-region step repeated over a fine
 * energy mesh for every symmetry, Eq. 1-2 its pole sum; the matching, K,
 * T and collision strengths are the standard R-matrix outer region the
 * paper's codes run, Sec. 2-3): for each energy E[e] (device, [M]) and each
 * of the n_sym symmetries, pole sum -> channel functions -> matching -> K
 * -> T, summing
 * (g/2)|T_ij|^2 over symmetries into omega (device,
 * [M][n_target*(n_target+1)/2], FP64, overwritten).  Target pair (t, u),
 * t <= u, sits at t*n_target - t(t-1)/2 + (u - t) of each energy's row.
 * status (device [M] int32, or NULL) receives the OR of the RM_E_* bits.
 * Every handle must have been loaded on the current device, and its target
 * levels must be < n_target.  Energies need no ordering.
 * Errors: RM_ERR_ARG, RM_ERR_STATE, RM_ERR_NOMEM, RM_ERR_HIP. */
int rm_sweep_energies(const rm_sym_t *syms, int32_t n_sym, int32_t n_target,
                      const double *E, int64_t M, const rm_opts *opts,
                      double *omega, int32_t *status, void *stream);

/* rm_sweep_energies without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * rm_sweep_energies.  Its workspace (the per-energy matching systems, the
 * channel slots, the pole-sum work tables and counters) lives in one static
 * device array of RM_NOALLOC_SCRATCH_BYTES, which every GPU the library
 * runs on holds until the process ends; the mesh is swept in chunks of as
 * many energies as that array holds (about 240 at 200 channels), so large
 * symmetries run with fewer energies in flight than rm_sweep_energies.
 * Differences: RM_FLAG_AUTOTUNE returns RM_ERR_ARG (timing allocates); the
 * pair form of the pole sum is used only where its products are already
 * resident (formed by an earlier allocating call), else the scaled-W
 * kernels; symmetries whose single energy (or whose tables and counters)
 * do not fit return RM_ERR_ARG.  The call synchronises `stream` once, after
 * copying its tables into the array, then enqueues the sweep.  Every call
 * on a GPU shares that GPU's array and leaves its contents behind: calls
 * that overlap on one GPU (other streams or host threads) race and must be
 * serialised by the caller. */
#define RM_NOALLOC_SCRATCH_BYTES (256u << 20)
int rm_sweep_energies_noalloc(const rm_sym_t *syms, int32_t n_sym,
                              int32_t n_target, const double *E, int64_t M,
                              const rm_opts *opts, double *omega,
                              int32_t *status, void *stream);

/* Captured sweep.  rm_plan_create validates like rm_sweep_energies, orders
 * the symmetries by cost, sizes the chunks and the workspace (owned by the
 * plan), builds the grouped pole-sum work tables (largest symmetries first),
 * and records the whole sweep -- per chunk one grouped pole-sum launch per
 * tile variant and one persistent matching launch covering every symmetry
 * and energy of the chunk -- into a hipGraph bound to E, omega and status.
 * rm_plan_execute replays it on `stream` (the caller may change the contents
 * of E between replays, not the pointers).  Replays of one plan must not
 * overlap.  rm_plan_create synchronises `stream` (autotuning and table
 * uploads); rm_plan_free synchronises the device.
 * rm_plan_info: energies per chunk, chunk count and the tile variant chosen
 * for each symmetry in kernel order (largest first).  A plan holds its
 * symmetries' descriptors as they were at rm_plan_create: rm_free or
 * rm_set_propagation on one of them releases device arrays that the plan's
 * graph still reads, so free the plan first; rm_set_gailitis takes effect
 * only in plans created after it. */
typedef struct rm_plan *rm_plan_t;
int rm_plan_create(const rm_sym_t *syms, int32_t n_sym, int32_t n_target,
                   const double *E, int64_t M, const rm_opts *opts,
                   double *omega, int32_t *status, void *stream,
                   rm_plan_t *out);
int rm_plan_execute(rm_plan_t plan, void *stream);
int rm_plan_info(rm_plan_t plan, int64_t *chunk, int32_t *n_chunks,
                 int32_t *variants, int32_t n_variants);
int rm_plan_free(rm_plan_t plan);

/* K-matrix of one symmetry at m energies (device E [m]): the pole sum of
 * Sec. 6 Eq. 1-2 matched at r = a (or at A, rm_set_propagation) to the
 * asymptotic channel functions.
 * K (device, [m][n][n] FP64, n = n_chan): the open-open block occupies the
 * leading n_open[e] x n_open[e] rows/columns (row-major, leading dimension
 * n), open channels in ascending input-channel order; other entries are 0.
 * n_open (device [m] int32) receives the open-channel counts.
 * R_opt (device [m][n][n] or NULL) receives R(E) in input-channel order.
 * status (device [m] or NULL) receives RM_E_* bits. */
int rm_kmatrix(rm_sym_t sym, const double *E, int64_t m, const rm_opts *opts,
               double *K, int32_t *n_open, double *R_opt, int32_t *status,
               void *stream);

/* Collision strengths (the Omega of the paper's Sec. 4-5 figures) from
 * given K-matrices (device, layout of rm_kmatrix):
 * T = 2iK(1 - iK)^-1 and omega[e][pair(t,u)] += (g/2)|T_ij|^2 over open
 * channels i of level t and j of level u (device omega [m][n_target*(
 * n_target+1)/2], accumulated, not cleared).  n_open and E must be the ones
 * rm_kmatrix used. */
int rm_collision_strengths(rm_sym_t sym, const double *K,
                           const int32_t *n_open, const double *E, int64_t m,
                           int32_t n_target, double *omega, void *stream);

/* Boundary R-matrix alone (Sec. 6, Eq. 1-2) at m energies: R (device,
 * [m][n][n], input-channel order).  opts->prec selects the arithmetic. */
int rm_rmatrix(rm_sym_t sym, const double *E, int64_t m, const rm_opts *opts,
               double *R, void *stream);

/* Channel functions at r = a, input-channel order: out (device [m][n][4]).
 * Open channel (E > e_i): (s, c, a s', a c') with s = k^-1/2 F_l(eta, ka),
 * c = k^-1/2 G_l, primes d/dr, eta = -z/k.  Closed channel: (e, a e', 0, 0),
 * the decaying Whittaker function W_{z/phi, l+1/2}(2 phi r) and a times its
 * r-derivative at r = a scaled to unit length.  status as above. */
int rm_channel_functions(rm_sym_t sym, const double *E, int64_t m,
                         double *out, int32_t *status, void *stream);

/* Stage timing (diagnostics).  rm_profile(1) clears the record and makes
 * every later call of this process bracket each kernel launch with HIP
 * events on the caller's stream; rm_profile(0) stops recording.
 * rm_profile_query synchronises on the recorded events and returns, for
 * stage 1 (pole sum), 2 (channel functions, matching, K, T, Omega), 3
 * (rm_plan_execute graph replays), 4 (the banded product of
 * rm_convolve_gaussian), 5 (the pass over Omega of
 * rm_effective_collision_strengths), 6 (the pass of
 * rm_group_collision_strengths), 7 (the outer-region propagation of
 * rm_set_propagation), 8 (the Jacobi sweeps of rm_inner_region, one record
 * per sweep) or 9 (its quadrature tables and Hamiltonian assembly), the
 * summed time in milliseconds and the
 * number of launches (stage 0 is kept for compatibility and stays empty).
 * Not thread-safe with concurrent sweeps while enabled. */
int rm_profile(int32_t enable);
int rm_profile_query(int32_t stage, double *total_ms, int64_t *launches);

/* ---- Learned adaptive mesh -------------------------------------------
 * The paper asks for millions of energies to resolve narrow resonances
 * (Sec. 3); a small network, trained on the device on cross sections the
 * sweep itself produces, predicts where resonances are so that a smaller
 * adaptive mesh can stand in for the uniform one.
 *
 * rm_mlp_create: dense network d_in -> width -> ... -> 1 with n_layers
 * layers (>= 2), SiLU between layers, linear output.  prec 0: BF16 operands
 * on the matrix cores with FP32 accumulation; prec 1: FP32 operands (debug).
 * Weights are initialised from `seed` (splitmix64, uniform He bounds).
 * Parameters form one flat FP32 array, layer by layer W_l [out][in] then
 * b_l [out]; rm_mlp_n_params gives its length.  get/set copy it from/to a
 * device array.  All data pointers are device pointers. */
typedef struct rm_mlp *rm_mlp_t;
int rm_mlp_create(int32_t d_in, int32_t width, int32_t n_layers, int32_t prec,
                  uint64_t seed, rm_mlp_t *out);
int rm_mlp_free(rm_mlp_t mlp);
int rm_mlp_n_params(rm_mlp_t mlp, int64_t *n);
int rm_mlp_get_params(rm_mlp_t mlp, float *dst, void *stream);
int rm_mlp_set_params(rm_mlp_t mlp, const float *src, void *stream);
/* Y [B] = net(X [B][d_in]). */
int rm_mlp_forward(rm_mlp_t mlp, const float *X, int32_t B, float *Y,
                   void *stream);
/* Mean squared error against target [B]; loss (device float, or NULL) and
 * the gradient of every parameter (kept for rm_mlp_adam_step and copied to
 * grad [n_params] when grad is not NULL). */
int rm_mlp_grad(rm_mlp_t mlp, const float *X, const float *target, int32_t B,
                float *loss, float *grad, void *stream);
/* One Adam update (Kingma & Ba 2015, bias-corrected) from the last gradient. */
int rm_mlp_adam_step(rm_mlp_t mlp, float lr, float beta1, float beta2,
                     float eps, void *stream);
/* Mesh from a density: dens [nw] (>= 0, device) on nw equal windows of
 * [lo, hi] is normalised, mixed with a uniform floor
 * (density = (1 - floor_frac) dens/sum + floor_frac/(hi - lo)), and M
 * energies are placed at the midpoints of M equal-mass intervals of its CDF
 * (piecewise linear inside a window).  E_out [M] ascending (device). */
int rm_mesh_from_density(const float *dens, int32_t nw, double lo, double hi,
                         double floor_frac, int64_t M, double *E_out,
                         void *stream);

/* ---- Outer-region propagation -------------------------------------------
 * The paper matches at r = a; for real targets the channels stay coupled
 * beyond a through the long-range multipole potentials of the target.
 * rm_set_propagation makes every later sweep of `sym` (rm_sweep_energies,
 * rm_kmatrix, plans) carry the R-matrix from a to A before matching there:
 * for r >= a, u'' = (W(r) - E) u with
 *   W_ij(r) = [e_i + l_i (l_i + 1)/r^2 - 2z/r] delta_ij
 *             + sum_{lam = 1..lmax} beta[lam - 1][i][j] / r^(lam + 1),
 * beta (host [lmax][n_chan][n_chan], input channel order, symmetric, Ry
 * a0^(lam+1)); n_sec sectors of equal width, W frozen at each sector's
 * midpoint and diagonalised once here (host Jacobi), the reduced R-matrix
 * u u'^-1 stepped exactly across each sector in its eigenbasis on the
 * device, R(A) matched to Coulomb / Whittaker functions at r = A (terms
 * beyond A dropped).  n_sec = 0 switches the propagation off.  rm_rmatrix
 * still returns R(a); rm_photoionization rejects propagated symmetries.
 * Synchronises `stream`.  Errors: RM_ERR_ARG (n_sec outside [0, 1e5], lmax
 * outside [0, 8], A not finite or <= a, beta null, not finite or not
 * symmetric), RM_ERR_STATE, RM_ERR_NOMEM, RM_ERR_HIP. */
int rm_set_propagation(rm_sym_t sym, double A, int32_t n_sec, int32_t lmax,
                       const double *beta, void *stream);

/* rm_set_gailitis keeps the multipole terms beyond A as well: the open-
 * channel solutions matched at A become the coupled asymptotic series of
 * Gailitis (J. Phys. B 9 (1976) 843), the standard outer-region expansion
 * (the paper says nothing of the region beyond a).  For the solution that
 * behaves as exp(i theta_j) in open channel j,
 *   u_i = g_ij exp(i theta_j),  g_ij = sum_p c^p_ij r^-p,
 *   theta_j = k_j r - eta_j ln(2 k_j r) - l_j pi/2 + sigma_j,
 * the coefficients follow from the equations above by powers of 1/r (a
 * three-term recurrence coupled through beta; channels of equal threshold
 * take the relation one order up); s = Im, c = Re of u / sqrt(k_j), and the
 * matching at A solves [C - R A C' | closed] [K; X] = R A S' - S with these
 * n x n_o matrices in place of the diagonal Coulomb functions (closed
 * channels keep their decaying Whittaker functions).  Each channel's series
 * is summed to its smallest term, at most max_terms terms: the first term
 * larger than the one before ends the sum unadded, a term below 1e-16 after
 * adding it; an energy whose first omitted term exceeds 1e-6 in some
 * channel gets RM_E_ASYM_NOCONV (A too small for its energies: near
 * thresholds, or between close thresholds, k r must be large against the
 * couplings).  max_terms = 0 switches the expansion off; rm_set_propagation
 * with n_sec = 0 switches both off.  Sweeps with solve_fp32 reject such
 * symmetries (the FP64 solve only).  Synchronises `stream`.  Errors:
 * RM_ERR_ARG (null handle, max_terms outside [0, 200]), RM_ERR_STATE (no
 * propagation set). */
int rm_set_gailitis(rm_sym_t sym, int32_t max_terms, void *stream);

/* ---- Photoionization ---------------------------------------------------
 * The photoionization runs of the paper (Sec. 2-3: one dipole per pair of
 * dipole-allowed symmetries, the outer-region module for photoionization;
 * Sec. 4-5: the N, O, Kr+, Xe+ and W3+ cross sections) reuse the
 * scattering solve at every energy with the bound-free dipole matrix
 * elements d_k = <psi_k | D | Psi_0> between each inner-region state k of a
 * final symmetry and the initial state (angular factors included).  Read
 * without radiation damping:
 *   g_i(E)  = (1/sqrt2) sum_k w_ik d_k / (E_k - E)   (a pole sum as Eq. 1)
 *   M_j     = sum_i u_ij'(a) g_i over every channel i, u_ij'(a) the radial
 *             derivative at r = a of channel i of the K-matrix solution j
 *             (s_i' delta_ij + c_i' K_ij open, e_i' X_ij closed)
 *   S(E)    = (1/pi) M (1 + K^2)^-1 M^T           (energy-normalised,
 *             summed over the final channels)
 *   sigma(E)= (4 pi^2 alpha a0^2 / 3) (E - e0) S(E)  in Mb, E and e0 in Ry,
 * summed over the symmetries passed.
 *
 * rm_load_dipoles: attach d (host [n_poles], finite, input pole order) to a
 * loaded symmetry (copied to its device; replaces an earlier vector after
 * synchronising `stream`).  Errors: RM_ERR_ARG, RM_ERR_STATE, RM_ERR_NOMEM,
 * RM_ERR_HIP. */
int rm_load_dipoles(rm_sym_t sym, const double *d, void *stream);

/* rm_load_widths: attach the radiative widths Gamma_k (host [n_poles], finite,
 * >= 0, Ry, input pole order) of the inner-region states to a loaded
 * symmetry, for the damped photoionization (replaces earlier widths after
 * synchronising `stream`).  Errors: RM_ERR_ARG, RM_ERR_STATE, RM_ERR_NOMEM,
 * RM_ERR_HIP.
 *
 * Radiation damping (the damped photoionization module of Sec. 3, Tables
 * 1-2; the paper gives no formula), read as the optical potential
 * -i sum_k (Gamma_k/2)|psi_k><psi_k|: the poles move to E_k - i Gamma_k/2,
 * so R and g become complex, and sigma is the flux into the open channels
 * of the driven solution of (E - H_eff) psi = D Psi_0 with outgoing waves:
 *   (diag(d1) - R_c diag(d2)) [alpha; beta] = -g_c,
 *   d1 = c + i s, d2 = a (c' + i s') (open), (e, a e') (closed),
 *   sigma(E) += (4 pi^2 alpha a0^2 / 3) (E - e0) (1/pi) sum_open |alpha_f|^2,
 * which equals the undamped sigma when every Gamma_k = 0.  Selected by
 * RM_FLAG_RADIATION_DAMPING in rm_photoionization's opts; it needs the FP64
 * pole sum and solve (prec = RM_PREC_FP64, solve_fp32 = 0, no autotuning or
 * pair products: RM_ERR_ARG otherwise) and widths on every symmetry.  The
 * complex system is solved as its real 2n x 2n form. */
int rm_load_widths(rm_sym_t sym, const double *gamma, void *stream);

/* rm_photoionization: sigma (device [M], overwritten) at the M energies E
 * (device, total energy of the final state on the thresholds' scale) for
 * the final symmetries `syms` (each with dipoles loaded) and the initial
 * state energy e0 (photon energy E - e0).  opts as for rm_sweep_energies
 * (the R-matrix pole sum may run mixed; the dipole pole sum is FP64).
 * status (device [M] or NULL): RM_E_* bits, RM_E_NO_OPEN below every
 * threshold (sigma 0 there).  Errors: RM_ERR_ARG (M < 0, e0 not finite,
 * null pointer, a symmetry without dipoles, bad opts), RM_ERR_STATE,
 * RM_ERR_NOMEM, RM_ERR_HIP. */
int rm_photoionization(const rm_sym_t *syms, int32_t n_sym, const double *E,
                       int64_t M, double e0, const rm_opts *opts,
                       double *sigma, int32_t *status, void *stream);

/* ---- Post-processing of Omega(E) on the mesh ------------------------
 * Omega arrays are energy-major [M][P] FP64 device arrays, P the number of
 * packed level pairs (t <= u, row-major over t) as rm_sweep_energies writes
 * them.  E (device [M]) must be ascending.
 *
 * rm_convolve_gaussian: the Gaussian smoothing applied before comparison
 * with measurements (Sec. 4 and 5, FWHM 4-124 meV in the paper's figures):
 *   out(E_i) = sum_j g_ij in(E_j) / sum_j g_ij,
 *   g_ij = exp(-(E_i - E_j)^2 / (2 s^2)) dE_j,  s = fwhm / (2 sqrt(2 ln 2)),
 * dE_j the trapezoid weights of the mesh (half intervals at its ends), the
 * sum cut at |E_i - E_j| <= 8 s.  fwhm in the units of E.  M = 1 copies the
 * input.  omega_out must not overlap omega_in.  The call is asynchronous on
 * `stream` (it allocates and frees 32 M bytes of stream-ordered workspace).
 * Errors: RM_ERR_ARG (M < 0, P < 1, fwhm not finite and > 0, null pointer,
 * in place), RM_ERR_NOMEM, RM_ERR_HIP. */
int rm_convolve_gaussian(const double *E, int64_t M, const double *omega_in,
                         int64_t P, double fwhm, double *omega_out,
                         void *stream);

/* rm_effective_collision_strengths: Maxwellian averages of every level pair
 * (t, u) at the nT temperatures kT (host [nT], > 0, units of E), the upper
 * level e = max(e_level[t], e_level[u]) (host [n_target]) and eps = E - e:
 *   Upsilon(kT) = int_0^inf Omega(eps) exp(-eps/kT) d(eps/kT),
 * Omega held constant from threshold to the first mesh point above e, the
 * trapezoid rule between mesh points, truncated at the last point (0 for a
 * pair whose upper level is at or above the mesh top).  Output upsilon
 * (device [P][nT], P = n_target (n_target + 1) / 2).  Host arrays are read
 * before the call returns; the call synchronises `stream`.
 * Errors: RM_ERR_ARG (M < 0, n_target < 1, nT < 0, kT not finite and > 0,
 * level energy not finite, null pointer), RM_ERR_NOMEM, RM_ERR_HIP. */
int rm_effective_collision_strengths(const double *E, int64_t M,
                                     const double *omega, int32_t n_target,
                                     const double *e_level, const double *kT,
                                     int32_t nT, double *upsilon,
                                     void *stream);

/* rm_group_collision_strengths: statistical averaging over the levels of
 * groups such as the fine-structure levels of a term (the level-averaged
 * cross sections of Sec. 5): out[i][pair(a, b)] (device [M][n_group (n_group
 * + 1) / 2]) is the sum of omega[i][pair(t, u)] over every level pair t <= u
 * with {group[t], group[u]} = {a, b}; group (host [n_target]) holds values in
 * [0, n_group).  The averaged cross section from group a follows as
 * pi Omega(a, b) / (g_a k^2), g_a the summed statistical weight of a.  The
 * call synchronises `stream`.
 * Errors: RM_ERR_ARG (M < 0, n_target < 1, n_group < 1, group index out of
 * range, null pointer), RM_ERR_NOMEM, RM_ERR_HIP. */
int rm_group_collision_strengths(const double *omega, int64_t M,
                                 int32_t n_target, const int32_t *group,
                                 int32_t n_group, double *out, void *stream);

/* ---- Inner region ----------------------------------------------------
 * The poles E_k and amplitudes w_ik of Eq. 1 come from the full
 * diagonalisation of each symmetry's inner-region Hamiltonian (Sec. 2-3:
 * every eigenpair, ScaLAPACK in the paper).  The atomic Hamiltonians are not
 * published; rm_inner_region diagonalises a multichannel model of the same
 * form on [0, a]:
 *   u_i'' = sum_j [(l_i (l_i + 1)/r^2 - 2z/r + e_i - E) delta_ij + U_ij] u_j,
 *   U_ij(r) = -depth_ij exp(-(r / range_ij)^2),
 * in the basis sqrt(2/a) sin(kappa_m r), kappa_m a = (m + 1/2) pi, m <
 * n_basis, per channel (index i n_basis + m), so u(0) = 0, u'(a) = 0 and the
 * kinetic part is diag(kappa_m^2); the potential's matrix elements by
 * n_quad-point Gauss-Legendre quadrature (0: n_basis + 48).  All eigenpairs
 * by blocked one-sided Jacobi on the device (round-robin pairs of 16-column
 * blocks; each pair's 32 x 32 Gram matrix diagonalised in LDS and its
 * rotation applied with FP64 MFMA); eigenvalues as Rayleigh quotients;
 * w_ik = sqrt2 u_ik(a), the convention of rm_load_poles.
 *
 * e_thr [n_chan], l [n_chan], depth and range [n_chan][n_chan] (symmetric,
 * range > 0): host.  E_pole (host [n_chan n_basis], ascending) and w (host
 * [n_chan][n_chan n_basis], columns in the order of E_pole; the sign of a
 * column and the basis of a degenerate eigenspace are arbitrary) are written
 * by the call, which synchronises `stream` after each sweep; sweeps and
 * rotations (host, each may be NULL) receive the sweeps taken and the
 * number of block-pair rotations applied over all of them.  Memory: about
 * 16 (n_chan n_basis)^2 + 8 (n_chan^2 + n_basis) n_quad bytes of device
 * workspace (the matrices, then the quadrature tables), allocated and freed
 * by the call.  Checked at D = n_chan n_basis = 8192 and 16384 by R(E)
 * between poles against a direct solve of (H - E) X = B^T, which tests the
 * eigenvectors and surface amplitudes, besides the eigenvalue sums.
 * Errors: RM_ERR_ARG (n_chan < 1, n_basis < 1, n_chan n_basis > 16384, a not
 * finite and > 0, z < 0, n_quad > 16384, n_chan^2 n_quad over 1e9 table
 * entries, l outside [0, 12], model arrays not
 * finite / not symmetric, null pointer), RM_ERR_NOMEM, RM_ERR_HIP,
 * RM_ERR_NUMERIC (no convergence in 40 sweeps; outputs hold the last
 * iterate). */
typedef struct {
  int32_t n_chan;
  int32_t n_basis;
  int32_t n_quad;
  double a;
  double z;
  const double *e_thr;
  const int32_t *l;
  const double *depth;
  const double *range;
} rm_inner_desc;
int rm_inner_region(const rm_inner_desc *desc, double *E_pole, double *w,
                    int32_t *sweeps, int64_t *rotations, void *stream);

/* rm_inner_region_batch: the inner-region step for `count` symmetries at
 * once (the paper diagonalises every symmetry's Hamiltonian).  Item b is
 * rm_inner_region(&descs[b], E_pole[b], w[b], &sweeps[b], &rotations[b]):
 * the same kernels and the same results, bit for bit, but the items run
 * concurrently, each on a stream of its own created on the caller's
 * current device (default priority) and driven by one of up to 8 host
 * threads, so that the kernels of small solves overlap.  E_pole and w are
 * host arrays of `count` host pointers sized as for rm_inner_region;
 * sweeps and rotations (host [count]) may be NULL.  `stream` is
 * synchronised first; the call returns when every item is done.
 * Workspace: each running item holds its own (at most 8 at a time).
 * Errors: RM_ERR_ARG (count < 0, null pointer), or the first failing
 * item's error with its index in the message (every item is attempted). */
int rm_inner_region_batch(const rm_inner_desc *descs, int32_t count,
                          double *const *E_pole, double *const *w,
                          int32_t *sweeps, int64_t *rotations, void *stream);

/* Message for the last non-RM_OK return on this thread ("" if none). */
const char *rm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RMATRIX_H */
