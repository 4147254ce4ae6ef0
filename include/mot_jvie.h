/*
 * mot_jvie.h -- C ABI of the MI355X (gfx950) library for the hot path of the
 * large-time-step marching-on-in-time current-density volume integral
 * equation (MOT-JVIE) solver for dielectric scattering of Kumar, Gerini and
 * van Beurden, "Large-Time-Step Operation in a Volume Integral Equation for
 * Dielectric Scattering".
 *
 * Problem (Sec. II): the TDJVIE of Eq. 1, discretized on a uniform voxel grid
 * with piecewise-constant spatial basis per Cartesian current component,
 * centre-point testing, Dirac temporal testing at t_n = n dt and the causal
 * quadratic-spline temporal basis (support [-dt, 2dt), T(0) = T(dt) = 1/2),
 * gives the MOT recursion of Eq. 3:
 *     Z0 J_n = E_n - sum_{k=1..ell} Z_k J_{n-k},   ell from Eq. 4,
 *     Z_k    = T(k dt) diag(eps_r) - diag(eps_r - 1) G_k,
 * so that Z0 = D - X G (Eq. 10) with D = diag(eps_r)/2, X = diag(eps_r - 1).
 * G_k is block Toeplitz (it depends only on voxel offsets); every product
 * with it is evaluated matrix-free through the circulant embedding and 3-D
 * FFTs of Eq. 11, assembled as Z0 J = D J - X (G J) (Eq. 12).
 *
 * Units: c0 = eps0 = h = 1 (h the voxel edge); times in h/c0.  The time step
 * is dt = alpha * dt_CFL with dt_CFL = h/(c0 sqrt 3), i.e. c0 dt / h = alpha/sqrt 3.
 *
 * Layouts (all arrays are caller-owned DEVICE memory, contiguous, at least
 * 16-byte aligned):
 *   voxel arrays (eps_r):            [nz][ny][nx], x fastest;
 *   current / field vectors (J, y):  [3][nz][ny][nx], component p in {x,y,z}
 *                                    slowest, then z, y, x.
 *   Green tables:                    [6][nz][ny][nx] over non-negative offsets
 *                                    (dz, dy, dx), components (xx,yy,zz,xy,xz,yz).
 *
 * Threading and streams: one context per stream; a context is not
 * thread-safe.  Every call enqueues on the context's stream and returns
 * without waiting, except where noted (mot_step and build_green_spectra read
 * scalars back).  No C++ exception crosses this interface.
 *
 * Errors: 0 on success, a negative MOT_E* code otherwise; mot_strerror()
 * names the code and mot_last_error() gives the detail of the last failure
 * on a context (HIP error strings included).
 */
#ifndef MOT_JVIE_H
#define MOT_JVIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MOT_OK = 0,
  MOT_EINVAL = -1,      /* bad shape, null pointer, unsupported length, bad enum */
  MOT_ENOMEM = -2,      /* device allocation failed */
  MOT_EHIP = -3,        /* a HIP call failed; see mot_last_error */
  MOT_ENOCONV = -4,     /* TFQMR reached max_iter; J_n holds the last iterate */
  MOT_EBREAKDOWN = -5,  /* TFQMR breakdown (rho or sigma exactly zero) */
  MOT_ENONFINITE = -6,  /* a NaN/Inf appeared in the right-hand side or the solution */
  MOT_ESTATE = -7       /* call out of order (e.g. no material or no spectra yet) */
};

typedef struct mot_ctx mot_ctx;

typedef enum {
  MOT_F64 = 0,          /* FFTs, spectra and Krylov vectors in FP64 */
  MOT_F32 = 1,          /* FFTs and spectral products in FP32 */
  MOT_F32_REFINED = 2   /* FP32 FFT products inside an FP64 iterative refinement */
} mot_precision;

typedef struct {
  int32_t nx, ny, nz; /* voxels per axis; nx even; 2*nx, 2*ny, 2*nz and nx must be
                         supported FFT lengths (products of 2, 3, 5 listed by
                         mot_length_supported) */
  int32_t alpha;      /* dt = alpha * dt_CFL, integer >= 1; 0 => use cdt */
  double cdt;         /* c0 dt / h when alpha == 0 (must be > 0) */
  int32_t nlags;      /* ell; 0 => Eq. 4 with p = 2 and R_max = sqrt(sum (N_i - 1/2)^2) */
  int32_t quad;       /* Gauss-Legendre nodes per quadrature piece, 0 => 20 (max 32) */
} mot_grid;

typedef struct {
  int32_t iters;        /* TFQMR iterations (two half steps each), all refinement sweeps */
  int32_t matvecs;      /* Z0 products in the solve, all precisions */
  int32_t matvecs_f64;  /* of which in FP64 */
  int32_t refinements;  /* outer refinement sweeps (MOT_F32_REFINED), else 0 */
  double relres;        /* final ||b - Z0 J_n|| / ||b|| evaluated in FP64 */
  double ms_lhs;        /* time of the solve (LHS of Eq. 6) */
  double ms_rhs;        /* time of the right-hand side: history update + assembly (RHS of Eq. 6) */
} mot_stats;

/* Modulated Gaussian plane wave of Eq. 7 and Eq. 8:
 *   E^i(r,t) = amp e exp(-tau^2/(2 sigma^2)) cos(2 pi f0 tau),
 *   tau = t - t0 - k.(r - r_c), r_c the grid centre, r the voxel centre. */
typedef struct {
  double e[3];   /* polarization */
  double k[3];   /* unit propagation direction */
  double f0, sigma, t0, amp;
} mot_pulse;

/* Create a context for `grid` with the given precision on `hip_stream`
 * (a hipStream_t; NULL = the default stream): one MOT system of Eq. 3 on the
 * voxel grid of Sec. II, with dt = alpha dt_CFL (Eq. 9) and ell lags (Eq. 4).  Allocates the FFT workspaces,
 * the Krylov vectors, the spectra and the history ring (ell spectra of past
 * currents: 3*(2nz)*(2ny)*(nx+1) complex each, FP64 for MOT_F64, else FP32).
 * Errors: MOT_EINVAL (shape, lengths, alpha/cdt), MOT_ENOMEM, MOT_EHIP. */
int mot_create(const mot_grid* grid, mot_precision prec, void* hip_stream, mot_ctx** out);

/* Release everything the context owns.  Accepts NULL. */
int mot_destroy(mot_ctx* ctx);

/* Sizes: out[0] = ell, out[1..3] = 2nx, 2ny, 2nz, out[4] = padded row
 * stride of the spectral buffers, out[5] = device bytes held by the context,
 * out[6] = steps taken since the last reset, and with n >= 8 out[7] = B, the
 * steps per history block (temporal blocking of the history sum), with
 * n >= 9 out[8] = the history scheme in use (1 or 2, mot_set_history_scheme).
 * Host array of n >= 7 entries. */
int mot_info(const mot_ctx* ctx, int64_t* out, int32_t n);

/* Operator precompute (Sec. II: Z_k for lags 0..ell; Sec. IV: spectra of the
 * circulant embedding).  For k = 0..ell evaluates G_k on the non-negative
 * octant of offsets (FP64 quadrature on the device), embeds each of its six
 * components on the doubled grid with the reflection signs, takes a 3-D FFT in
 * FP64 and keeps the real part on the octant of frequencies, scaled by
 * 1/(8 nx ny nz).  Blocks until done.  Errors: MOT_EHIP. */
int build_green_spectra(mot_ctx* ctx);

/* Largest |imaginary part| met while building the spectra (they are real up
 * to rounding because every component is even or odd-odd per axis). */
double mot_spectra_imag(const mot_ctx* ctx);

/* Set eps_r per voxel (device pointer, nx*ny*nz FP64, copied): the relative
 * permittivity eps(r)/eps0 of Eq. 1 (Sec. II), piecewise constant on the
 * voxels; it sets D = diag(eps_r)/2 and X = diag(eps_r - 1) of Eq. 10.  Voxels
 * with eps_r = 1 carry no current (the contrast current of Eq. 2 vanishes
 * there).  Errors: MOT_EINVAL. */
int mot_set_material(mot_ctx* ctx, const double* eps_r);

/* y = Z0 J (Eq. 12) with the FFT product of Eq. 11 (D = diag(eps_r)(1/2 +
 * d0) with the regularization of mot_set_regularization, d0 = 0 by default).
 *   dtype MOT_F64:         J, y FP64 device vectors, FP64 transforms;
 *   dtype MOT_F32:         J, y FP32 device vectors, FP32 transforms;
 *   dtype MOT_F32_REFINED: J, y FP64 device vectors, FP32 transforms (the
 *                          inner operator of the refined solver).
 * J and y must not overlap.  Errors: MOT_EINVAL, MOT_ESTATE, MOT_EHIP. */
int z0_matvec(mot_ctx* ctx, const void* J, void* y, mot_precision dtype);

/* Green-convolution only: y = (G_k J) for lag k (same dtypes as z0_matvec;
 * k = 0 uses the present-time spectra, k >= 1 the history spectra, whose
 * precision is the ring's).  Test entry point for the history operators. */
int gk_matvec(mot_ctx* ctx, int32_t k, const void* J, void* y, mot_precision dtype);

/* Push J_n (FP64 device vector) into the history ring and prepare the
 * history right-hand side of the next step (Eq. 3, Eq. 6 RHS),
 *   h_{n+1} = -sum_{k=1..ell} Z_k J_{n+1-k}
 *           = -(1/2 + d1) eps_r J_n - d2 eps_r J_{n-1} + (eps_r - 1) sum_{k=1..ell} G_k J_{n+1-k},
 * using the spectra of past currents (each current is transformed once).
 * The spectral sums are blocked in time: every B steps (B = 8, halved while
 * B > ell) one pass over the ring accumulates the contributions of all
 * stored currents to the next B right-hand sides; the steps in between add
 * only their newest lags.  With the history scheme of FFTs in time (see
 * mot_set_history_scheme) the lags that reach back before the current block
 * of 32 steps are applied once per such block in the frequency domain of
 * time, and the blocked pass covers the current block's currents only.
 * Errors: MOT_ESTATE, MOT_EHIP. */
int history_update(mot_ctx* ctx, const double* J_n);

/* Copy the prepared history right-hand side (FP64, 3N) to `out` (device). */
int mot_get_history_rhs(mot_ctx* ctx, double* out);

/* out = (eps_r - 1) d/dt E^i(r_m, t) at every voxel centre (the tested
 * excitation of Eq. 1), FP64 device vector of 3N. */
int mot_excitation(mot_ctx* ctx, const mot_pulse* pulse, double t, double* out);

/* One MOT step (Eq. 3): b = einc + h_n, solve Z0 J_n = b by TFQMR from
 * J = 0 to ||b - Z0 J_n|| <= tol ||b|| (true residual, FP64), then
 * history_update(J_n) and n += 1.  b = 0 gives J_n = 0 after 0 iterations.
 * einc, J_n: FP64 device vectors of 3N (distinct).  `stats` may be NULL;
 * with stats the call waits for the step to finish (it times the solve and
 * the right-hand side), without it the history update is still in flight
 * when it returns.
 * Errors: MOT_ENOCONV (J_n = last iterate, history still advanced),
 * MOT_EBREAKDOWN, MOT_ENONFINITE, MOT_ESTATE, MOT_EHIP. */
int mot_step(mot_ctx* ctx, const double* einc, double* J_n, double tol, int32_t max_iter, mot_stats* stats);

/* Statistics of the context's last mot_step (host copy, no device wait):
 * iterations, products, refinements and the final residual of Eq. 3's
 * solve; ms_lhs and ms_rhs are -1 when that step was called without
 * stats.  Errors: MOT_EINVAL (NULL). */
int mot_last_stats(const mot_ctx* ctx, mot_stats* stats);

/* on = 1: each TFQMR iteration of mot_step is replayed from a HIP graph
 * (captured on first use, per vector precision, operator and whether it
 * carries the true-residual check; the capture uses a stream of the
 * context's own, the replay the context's stream).
 * on = 2 (MOT_F32_REFINED without an initial guess): the first refinement
 * sweep of a step, i.e. the inner FP32 TFQMR with a fixed number of
 * iterations behind the convergence gates (one more than the most that the
 * first sweeps of the last 8 steps needed) and its FP64 residual, is one
 * graph replay, followed by one read of the residual; further sweeps, and
 * the first step after the mode is set, run launch by launch.  The graph is
 * captured again when that iteration count, the tolerance or the operator
 * changes.  The currents are those of on = 0, bit for bit.
 * Timing (mot_profile) uses the launch-by-launch path.  Errors: MOT_EINVAL. */
int mot_set_graphs(mot_ctx* ctx, int32_t on);

/* Batch of independent scatterers: one MOT step (as mot_step) of each of the
 * `count` contexts, run by `nthreads` host threads so that contexts created
 * on different streams overlap on the GPU (streams share the device's few
 * hardware queues: about 8 threads reach the best rate for 32 small grids).  einc[i], J_n[i]: the i-th
 * context's vectors; stats (may be NULL: those of mot_last_stats, without
 * LHS/RHS times) and status (required) are arrays of count.  Every context must be distinct (a context is not thread-safe).
 * Returns MOT_OK or the first non-OK status; status[i] holds each one.
 * Errors: MOT_EINVAL, and those of mot_step. */
int mot_step_batch(mot_ctx* const* ctxs, int32_t count, const double* const* einc, double* const* J_n, double tol,
                   int32_t max_iter, mot_stats* stats, int32_t* status, int32_t nthreads);

/* ---- Tile shapes of the FFT passes (Eq. 11 products) and their autotuner.
 *
 * Each pass of the Green products has two tile shapes, variant 0 (the
 * default) and variant 1:
 *   knob 0, x passes:        NP rows per workgroup, or 3 (NP/4) whole voxel
 *                            rows of all three components;
 *   knob 1, y passes:        NP kx columns per workgroup, or 2 NP when that
 *                            fits a workgroup (else NP/2);
 *   knob 2, history z passes: W kx columns per workgroup, or W/2;
 *   knob 3, fused z pass:    W kx columns per workgroup, or W/2.
 * Every variant computes the same sums in the same order: results are bit-identical
 * across variants.  The knobs are held per compute precision:
 * variants[4 p + k], p = 0 for the FP32 products, 1 for FP64.
 *
 * mot_set_variants: variants (host, 8 entries of 0 or 1).  Built Z0 spectra
 *   are rewritten in the fused z pass's new tile layout; captured iteration
 *   graphs are dropped.  Errors: MOT_EINVAL (NULL, a value other than 0 or 1).
 * mot_get_variants: the current variants into `variants` (host, 8 entries).
 * mot_autotune: times both variants of each knob on this context's grid and
 *   keeps the faster (variant 1 only when it is faster by more than 2%):
 *   knobs 0, 1, 3 by Z0 products in both precisions, knob 2 by the history z
 *   passes in the history precision.  Each timing is the least over three
 *   trials of `reps` calls (reps = 0: 20).  ms (host, optional, 16 entries):
 *   ms[2 (4 p + k) + v] = milliseconds per call of variant v, -1 where not
 *   timed.  Needs material and spectra, and a context at step 0 (a fresh
 *   context or after mot_reset): it uses the history spectrum buffer and
 *   leaves it zeroed.  Synchronises the context's stream.
 *   Errors: MOT_EINVAL (reps < 0), MOT_ESTATE, MOT_EHIP. */
int mot_set_variants(mot_ctx* ctx, const int32_t* variants);
int mot_get_variants(const mot_ctx* ctx, int32_t* variants);
int mot_autotune(mot_ctx* ctx, int32_t reps, double* ms);

/* Initial guess of the MOT_F32_REFINED solve (not in the paper; the solution
 * still meets the same true-residual test): with k > 0 the context keeps the
 * solutions J_i of its last k steps and Z0 J_i (the product its last FP64
 * residual computes anyway) and starts each solve from x0 = sum_i c_i J_i,
 * c the least-squares fit of the right-hand side by the Z0 J_i, so that
 * r0 = b - sum_i c_i Z0 J_i costs no product.  Uses 2k FP64 vectors of 3N,
 * allocated on first use.  Default k = 0 (off).  The stored pairs are dropped by mot_reset, mot_set_step,
 * mot_set_material, build_green_spectra, a change of mot_set_adjoint and this
 * call.  Errors: MOT_EINVAL (k outside 0..8, or k > 0 for another precision). */
int mot_set_predictor(mot_ctx* ctx, int32_t k);

/* Regularized interaction matrices in the delta-notation of Sec. II
 * (Z^delta_n = Z_n + delta_n I; the paper runs with delta_n = 0).  Here
 * delta_n = d_n diag(eps_r) for n = 0, 1, 2 and 0 beyond: the constitutive
 * term eps_r J of Eq. 1 is weighted (1/2 + d0, 1/2 + d1, d2) on (J_n,
 * J_{n-1}, J_{n-2}) instead of the spline's (1/2, 1/2, 0).  With weights
 * that sum to 1 (d0 + d1 + d2 = 0) the static response is unchanged; a
 * difference such as (d, -d, 0) or (d/2, -d, d/2) damps the current pattern
 * that alternates in sign from step to step, which the spline does not see
 * at the testing instants.  Z0 = diag(eps_r)(1/2 + d0) - X G_0 in z0_matvec,
 * mot_step and the adjoint calls; the history right-hand side carries
 * -(1/2 + d1) eps_r J_n - d2 eps_r J_{n-1} (d2 != 0 keeps one more current,
 * 3N FP64, allocated by this call and zeroed by mot_reset).  Default all
 * zero (the paper's operator).  May be called at any time; the next step
 * uses it.  Drops captured iteration graphs and the initial-guess pairs.
 * Errors: MOT_EINVAL (NULL, a value not finite, 1/2 + d0 <= 0), MOT_ENOMEM. */
int mot_set_regularization(mot_ctx* ctx, double d0, double d1, double d2);

/* TFQMR (the solver of Eq. 3 at every step, Sec. II) breaks down when
 * rho = r~^T r or sigma = r~^T A u vanishes.  By default only an exact zero
 * counts (t = 0); with t > 0 the solver also stops when |rho| or |sigma| is at
 * most t |b|^2 (|b| of the solve's right-hand side): a near-breakdown guard,
 * and the way to make the breakdown exit happen on purpose (failure
 * injection: a huge t ends every solve with MOT_EBREAKDOWN at its first
 * reduction, mot_step still advances the history).  Applies from the next
 * solve.  Errors: MOT_EINVAL (NULL, t negative or not finite). */
int mot_set_breakdown_tolerance(mot_ctx* ctx, double t);

/* How history_update evaluates sum_k Lambda_k J^_{n+1-k}, the history
 * right-hand side that dominates at small time steps (Sec. III-A, small
 * time-step regime; Sec. III-B evaluates it with an FFT-based
 * delayed-history scheme):
 *   1  per-lag multiply-accumulate over all ell lags, blocked in time (B = 8);
 *   2  FFTs in time: the steps are grouped in blocks of S = 32; at the first
 *      push of a block the lags reaching back into each earlier block m are
 *      applied as one product per frequency of a length-2S transform in time
 *      (the spectra of the lag segments Lambda_{(m-1)S+1..(m+1)S-1} are
 *      computed once, with the spectra, from the stored Lambda_k), and the
 *      lags inside the current block stay with the blocked pass of scheme 1.
 *      The same sums up to rounding; the work per step drops from O(ell)
 *      multiply-adds per frequency to O((ell / S) log S).  Needs an FP32 ring
 *      (precision MOT_F32 or MOT_F32_REFINED) and ell >= 32; it holds
 *      (ell - 1) / 32 + 1 transformed lag segments (33 complex frequencies
 *      of the 6 components each, FP32) and 32 right-hand-side spectra;
 *   0  the library's choice (the default): 2 when possible and ell >= 128.
 * A change applies from the next push on (a block of 32 steps that has
 * begun finishes with scheme 1).  mot_info reports the scheme in use.
 * Errors: MOT_EINVAL (NULL, scheme not 0..2, scheme 2 not possible),
 * MOT_ENOMEM. */
int mot_set_history_scheme(mot_ctx* ctx, int32_t scheme);

/* Address form of the FP32 blocked history multiply-accumulate (a check of
 * the library against itself, not an operation of the method).  By default
 * its loads take 32-bit byte offsets from a per-slot base whenever a ring
 * slot (three spectra) and a lag of Lambda (six components) each fit in
 * 4 GiB, and 64-bit addresses on larger grids; on = 1 forces the 64-bit form
 * on any grid, on = 0 restores the default.  The two forms give the same
 * sums bit for bit.  Applies from the next push on.
 * Errors: MOT_EINVAL (NULL, on not 0 or 1). */
int mot_set_wide_offsets(mot_ctx* ctx, int32_t on);

/* Start a new march of Eq. 3: n = 0, history ring and history right-hand
 * side zeroed (J_{n<0} = 0: the causal start of the recursion). */
int mot_reset(mot_ctx* ctx);

/* Set the step counter to n >= 0 without touching the history ring or the
 * history right-hand side.  After mot_reset this starts the march at step n
 * with J_m = 0 for every m < n (all ell ring slots count as filled), which
 * is the steady-state cost of every later step. */
int mot_set_step(mot_ctx* ctx, int64_t n);

/* Evaluate G_k on the octant of offsets into `out` ([6][nz][ny][nx] FP64,
 * device), exactly as build_green_spectra does.  Entries outside the causal
 * region of lag k are exact zeros. */
int mot_green_table(mot_ctx* ctx, int32_t k, double* out);

/* Kernel timing.  When enabled, every launch of the hot path is bracketed by
 * a pair of HIP events on the context's stream and its duration is added to
 * one of MOT_PROF_NCLASS classes:
 *   class = 2*kind + (FP64 ? 1 : 0), kind: 0 x forward, 1 y forward,
 *   2 z fused (forward, Lambda, inverse), 3 y inverse, 4 x inverse + Eq. 12
 *   epilogue, 5 z forward (history spectra), 6 history multiply-accumulate
 *   over all old slots (start of a block of steps), 7 z inverse (history),
 *   8 Krylov vector/reduction kernels (FP64: odd class), 9 excitation,
 *   10 history multiply-accumulate of the newest lags inside a block,
 *   11 history far lags by FFTs in time (start of a block of 32 steps).
 * mot_profile_read copies the accumulated milliseconds and launch counts of
 * the n = MOT_PROF_NCLASS classes to host arrays, then clears them (it
 * waits for the stream).  Timing adds a few microseconds per launch. */
#define MOT_PROF_NCLASS 24
int mot_profile(mot_ctx* ctx, int32_t enable);
int mot_profile_read(mot_ctx* ctx, double* ms, int64_t* counts, int32_t n);
/* Restrict timing to the kinds whose bit is set in kind_mask (bit k = kind
 * k above; default: all).  Untimed launches carry no events, so a narrow
 * mask keeps the timing overhead off the rest of the step.
 * Errors: MOT_EINVAL (negative mask). */
int mot_profile_kinds(mot_ctx* ctx, int32_t kind_mask);

/* ---- Adjoint march and permittivity gradient (Eq. 1, Eq. 10 structure).
 *
 * Every G_k is a symmetric matrix (G_k(-d) = G_k(d), symmetric 3x3 blocks),
 * so the transposed interaction matrices are
 *   Z_k^T = T(k dt) diag(eps_r) - G_k diag(eps_r - 1):
 * the contrast acts on the input.  The transpose of the march
 * sum_k Z_k J_{n-k} = E_n is solved backwards in time,
 *   Z0^T lam_n = g_n - (eps_r/2) lam_{n+1} + sum_{k>=1} G_k ((eps_r - 1) lam_{n+k}),
 * with the same ring, blocking and solver as the forward march.
 *
 * Far field (reading; not in the paper): the current radiates through the
 * retarded potential of Eq. 1; in the unit direction r, with the factor
 * 1/(4 pi R) and the delay R dropped and samples at tau_j = j dt,
 *   e_j = -(1/(4 pi dt)) (I - r r^T) sum_m sum_n J_{m,n} T'(j - n + r . r_m / dt),
 * r_m the voxel centre relative to the grid centre, T' the derivative of the
 * temporal basis in step units.  For W = dt sum_j |e_j|^2 the adjoint sources
 * are g_n = mot_farfield_adjoint(2 dt e) and
 *   dW/d eps_m = sum_n lam_n(m) . (d_t E^i(r_m, t_n) - w0 J_n(m) - w1 J_{n-1}(m)
 *                                  - w2 J_{n-2}(m) + u_n(m)),
 * (w0, w1, w2) = (1/2 + d0, 1/2 + d1, d2) with the regularization's d,
 * u_n = sum_{k=0..ell} G_k J_{n-k} = (mot_history_gfield read just before
 * step n) + gk_matvec(0, J_n). */

/* on = 1: the context's solver and history use Z_k^T (mot_step then takes
 * an adjoint step: einc is g_n, J_n receives lam_n, steps run backwards in
 * time); on = 0: the forward operators.  Call mot_reset after switching.
 * Errors: MOT_EINVAL. */
int mot_set_adjoint(mot_ctx* ctx, int32_t on);

/* y = Z0^T v = (1/2 + d0) eps_r v - G_0 ((eps_r - 1) v), dtypes as z0_matvec.
 * Errors: MOT_EINVAL, MOT_ESTATE, MOT_EHIP. */
int z0t_matvec(mot_ctx* ctx, const void* v, void* y, mot_precision dtype);

/* out (FP64 device, 3N, not the context's own buffers) = the Green part of
 * the prepared history for the coming step n: sum_{k>=1} G_k J_{n-k}
 * (adjoint context: sum_{k>=1} G_k ((eps_r - 1) lam_{n+k})).  Zero after
 * mot_reset.  Errors: MOT_EINVAL, MOT_ESTATE, MOT_EHIP. */
int mot_history_gfield(mot_ctx* ctx, double* out);

/* e (FP64 device, [nj][3]) = far-field samples j = j0 .. j0+nj-1 of the
 * current history Jhist (FP64 device, [nsteps][3N], step n at n*3N) and, if
 * `energy` (FP64 device scalar) is not NULL, energy = dt sum_j |e_j|^2.
 * rhat: host array of 3 (normalized by the library; zero is an error).
 * Deterministic (fixed partial sums).  1 <= nj <= 65535.
 * Errors: MOT_EINVAL, MOT_ENOMEM, MOT_EHIP. */
int mot_farfield(mot_ctx* ctx, const double* Jhist, int32_t nsteps, const double* rhat, int32_t j0, int32_t nj,
                 double* e, double* energy);

/* mot_farfield for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same samples and energy, bit for bit, with the block partials in a
 * static device array of the library (6 MiB per GPU, held until the process
 * ends) instead of a context buffer grown on first use.  Allocates nothing.
 * 1 <= nj <= 1024 (larger nj: MOT_EINVAL).  The array belongs to the calling
 * thread's current device, which must be the context's.  Every call on one
 * GPU shares that array: calls that overlap on one GPU (other streams or
 * threads) race.  Nothing in it needs to start at zero (each call writes the
 * partials it reads).  Errors: MOT_EINVAL, MOT_EHIP. */
int mot_farfield_static(mot_ctx* ctx, const double* Jhist, int32_t nsteps, const double* rhat, int32_t j0,
                        int32_t nj, double* e, double* energy);

/* g_n (FP64 device, 3N) = scale * (transpose of mot_farfield applied to the
 * weights w (FP64 device, [nj][3]) for step n): scale times the derivative
 * of sum_j w_j . e_j with respect to J_n (w = e, scale = 2 dt gives
 * dW/dJ_n).  Errors: MOT_EINVAL, MOT_EHIP. */
int mot_farfield_adjoint(mot_ctx* ctx, const double* w, int32_t j0, int32_t nj, const double* rhat, double scale,
                         int64_t n, double* g_n);

/* grad[m] += sum_p lam_n[p,m] (d_t E^i_p(r_m, t) - w0 J_n[p,m] - w1 J_prev[p,m] - w2 J_prev2[p,m]
 *                               + uh_n[p,m] + u0_n[p,m])
 * for every voxel m (w as above): the step-n term of dW/d eps with
 * u_n = uh_n + u0_n split into its history part (mot_history_gfield before
 * step n) and its present part (gk_matvec(0, J_n)).  FP64 device vectors:
 * lam_n, J_n, J_prev (J_{n-1}), J_prev2 (J_{n-2}), uh_n, u0_n of 3N, grad of
 * N; J_prev and J_prev2 may be NULL where the step does not exist.
 * Errors: MOT_EINVAL, MOT_EHIP. */
int mot_adjoint_gradient(mot_ctx* ctx, const mot_pulse* pulse, double t, const double* lam_n, const double* J_n,
                         const double* J_prev, const double* J_prev2, const double* uh_n, const double* u0_n,
                         double* grad);

/* Host helpers (no GPU needed). */
int32_t mot_nlags(const mot_grid* grid);           /* ell of Eq. 4 (reading above), or < 0 */
int64_t mot_zk_nnz(const mot_grid* grid, int32_t k); /* nonzeros of Z_k with dyad weights 3/3/5/9, or < 0 */
int32_t mot_length_supported(int32_t n);           /* 1 if n is a supported FFT length */

const char* mot_strerror(int status);
const char* mot_last_error(const mot_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MOT_JVIE_H */
