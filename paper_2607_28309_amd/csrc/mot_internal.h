// Internal state and launchers of the MOT-JVIE library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/mot_jvie.h"
#include "fft_passes.h"

namespace motimpl {

// Krylov scalar slots kept in device memory (FP64).
enum Slot {
  S_RHO = 0,
  S_ALPHA,
  S_THETA,
  S_TAU,
  S_ETA,
  S_BETA,
  S_SIGMA,
  S_W2,
  S_RHONEW,
  S_B2,
  S_FLAG,
  S_DCOEF,
  S_R2,
  S_TAU0,
  S_X2,
  S_ETAP,  // coefficient of an x update still to be applied (x += etap d)
  S_BOUND_ONLY,  // 1: the quasi-residual bound ends the solve (no true residual)
  S_OB2,         // |b|^2 of the refined solve's FP64 right-hand side
  // device-side convergence state of a solve (S_CHECK must follow S_DONE:
  // the launch gates read the pair)
  S_DONE,
  S_CHECK,
  S_ITER,
  S_MAXIT,
  S_TOL,
  S_BNORM,
  S_STATUS,
  S_RELRES,
  S_NMV,
  S_BDTOL,  // near-breakdown tolerance: |rho| or |sigma| <= S_BDTOL |b|^2 (0: exact zero only)
  S_NSLOT
};
static_assert(S_CHECK == S_DONE + 1, "gates read done and check as a pair");

constexpr int RED_BLOCKS = 1024;   // fixed partial count: deterministic reductions
constexpr int RED_THREADS = 256;

// ---- green.hip
hipError_t launch_green(double* out, int nx, int ny, int nz, int k, int alpha, double L, int nq,
                        hipStream_t s);
hipError_t launch_embed(const double* goct, double* E, int comp, int nx, int ny, int nz, hipStream_t s);
int compress_blocks(int nx, int ny, int nz);
// w64 / w32 = 0: [comp][kzc][kyc][kxs] (history lags); > 0: the fused z
// pass's tile layout (motfft::lam_tile_offset) with tiles of that many columns
hipError_t launch_compress(const void* spec, double* lam64, float* lam32, double* imax, int comp, int nx,
                           int ny, int nz, int kxs, double scale, int w64, int w32, hipStream_t s);

// ---- krylov.hip (vectors of length n, element type V = float or double)
using motfft::Gate;
// Scalar recurrence applied by the reduction that produced scal[slot].
enum Post { POST_NONE = 0, POST_INIT, POST_ALPHA, POST_HALF0, POST_HALF1, POST_BETA, POST_RESID };
// Sum of nparts partials (RED_BLOCKS for the vector kernels here, the
// workgroup count for sums fused into the x passes) into scal[slot]; with
// mirror (pinned host memory), the S_NSLOT scalars are also written there,
// whether or not the gate is open.
hipError_t reduce_post(const double* partials, double* scal, int slot, int post, hipStream_t s, Gate g = Gate{},
                       int nparts = RED_BLOCKS, double* mirror = nullptr);
// Two sums at once (partials[0, nparts) and [stride, stride + nparts)), then
// post1 and post2 in that order.
hipError_t reduce_post2(const double* partials, double* scal, int slot1, int post1, int slot2, int post2,
                        hipStream_t s, Gate g, int nparts, int stride);
// Start of a solve: tol, max_iter and the convergence state (iteration 0, not
// done); bound_only: stop when the quasi-residual bound passes (for inner
// solves whose result an outer residual checks).
hipError_t solver_setup(double* scal, double tol, int max_iter, hipStream_t s, bool bound_only = false,
                        double breakdown_tol = 0.0);
// x += scal[slot] d
template <typename V> hipError_t vec_axpy_scal(V* x, const V* d, const double* coef, long long n, hipStream_t s);
// Initial guess from earlier solutions (at most PRED_MAX pairs J_i, Z0 J_i).
constexpr int PRED_MAX = 8;
struct DotSet {
  const double* u[2];        // u[0] = b; u[1] = the newest Z0 J (may be null)
  const double* w[PRED_MAX]; // the stored Z0 J_i
  int nu, nw;
};
// Dots u_j . w_i (index j nw + i), then u_0 . u_0 (index nu nw): one pass
// over the vectors, RED_BLOCKS partials per dot, then one block per dot
// sums them in a fixed order into out (device).
hipError_t multidot(const DotSet& ds, long long n, double* partials, double* out, hipStream_t s);
struct Combo {
  const double* J[PRED_MAX];
  const double* Z[PRED_MAX];
  double c[PRED_MAX];
  int k;
};
// x0 = sum_i c_i J_i, r0 = b - sum_i c_i Z_i
hipError_t pred_combine(const Combo& cb, const double* b, double* x0, double* r0, long long n, hipStream_t s);
// x *= rs per voxel (x: components of nvox values each)
template <typename V> hipError_t vec_scale_voxel(V* x, const V* rs, long long n, long long nvox, hipStream_t s);
template <typename V> hipError_t dot_partial(const V* a, const V* b, long long n, double* partials, hipStream_t s);
template <typename V> hipError_t vec_sub(const V* a, const V* b, V* out, long long n, double* partials,
                                         hipStream_t s, Gate g = Gate{});  // out = a - b, partials of |out|^2
template <typename V> hipError_t vec_zero(V* a, long long n, hipStream_t s);
hipError_t vec_add64(const double* a, const double* b, double* out, long long n, double* partials,
                     hipStream_t s);  // out = a + b, partials of |out|^2
hipError_t vec_copy(const double* a, double* out, long long n, hipStream_t s);
template <typename V> hipError_t tfqmr_init(const V* r0, V* w, V* u, V* rt, V* d, V* x, long long n, hipStream_t s);
// x64 (= or +=) (x32 + coef d) rs per voxel (3 components of nvox voxels);
// coef may be null (no update)
hipError_t finish_f2d(const float* x32, const float* d, const double* coef, const float* rs, double* x64,
                      long long nvox, bool acc, hipStream_t s);
// the same start from an FP64 r0 rounded to FP32, with |r0|^2 partials
hipError_t tfqmr_init_d2f(const double* r0, float* w, float* u, float* rt, float* d, float* x, long long n,
                          double* partials, hipStream_t s);
template <typename V> hipError_t tfqmr_v0(V* v, const V* au, const V* rt, long long n, double* partials,
                                          hipStream_t s, Gate g);

// ---- history.hip: history multiply-accumulate (ring slot t mod nl holds J^_t)
// out = init + sum_{j=1..nrec} Lambda_j J^_{n+1-j}   (init may be null)
hipError_t launch_mac_recent(const void* ring, const void* lamh, const void* init, void* out, int f64, int nl,
                             long long n, int nrec, int nx, int ny, int nz, int kxs, hipStream_t s);
// P_b = init_b + sum_{m<nold} Lambda_{m+b} J^_{n0-m}, b = 1..B: P_1 -> out0,
// P_b -> pblk + (b-2) slots; init_b = iblk + (b-1) slots (zero if iblk is null).
// wide != 0: 64-bit addresses also where 32-bit buffer offsets would do.
hipError_t launch_mac_block(const void* ring, const void* lamh, void* out0, void* pblk, const void* iblk, int f64,
                            int B, int nl, long long n0, int nold, int nx, int ny, int nz, int kxs, hipStream_t s,
                            int wide = 0);
// History by FFTs in time (FP32 ring): time blocks of TF_S steps, transforms
// of length 2 TF_S.  tfft_blocks(nl) spectra K_m (m = 1..M) of the lag
// segments Lambda_{(m-1)S+d}, d = 1..2S-1, each at the S+1 frequencies
// w = 0..S, [m-1][component][w][octant point] complex FP32.
constexpr int TF_S = 32;
inline int tfft_blocks(int nl) { return (nl - 1) / TF_S + 1; }
hipError_t launch_tfft_prep(const float* lamh, void* K, int nl, int nx, int ny, int nz, int kxs, hipStream_t s);
// far[i] = sum over the time blocks before step n + 1 of the lags they reach,
// for the S right-hand sides of steps n + 1 + i, i = 0..S-1 (n a multiple of
// S; ring slots older than n - nl + 1 or before step 0 read as zero)
hipError_t launch_tfft_far(const void* ring, const void* K, void* far, int nl, long long n, int nx, int ny, int nz,
                           int kxs, hipStream_t s);

// ---- mot_api.hip: excitation
hipError_t launch_einc(const mot_pulse* p, double t, const double* eps, double* out, int nx, int ny, int nz,
                       hipStream_t s);

// Centre of voxel m ([z][y][x], x fastest) relative to the grid centre, units of h.
__device__ __forceinline__ void voxel_centre(long long m, int nx, int ny, int nz, double& x, double& y, double& z) {
  const int ix = (int)(m % nx), iy = (int)((m / nx) % ny), iz = (int)(m / ((long long)nx * ny));
  x = ix + 0.5 - 0.5 * nx;
  y = iy + 0.5 - 0.5 * ny;
  z = iz + 0.5 - 0.5 * nz;
}

// Scalar factor of d/dt E^i at (x, y, z), time t (Eq. 7, Eq. 8): the field
// derivative is this times the polarization p.e.
__device__ __forceinline__ double incident_dt(const mot_pulse& p, double t, double x, double y, double z) {
  const double tau = t - p.t0 - (p.k[0] * x + p.k[1] * y + p.k[2] * z);
  const double w = 2.0 * 3.14159265358979323846 * p.f0;
  const double env = exp(-tau * tau / (2.0 * p.sigma * p.sigma));
  return p.amp * env * (-(tau / (p.sigma * p.sigma)) * cos(w * tau) - w * sin(w * tau));
}

// ---- adjoint.hip: far field of a current history, its transpose, gradient
// Far-field geometry: unit direction r, projection P = I - r r^T, step dt.
struct FarGeom {
  double r[3];
  double P[9];
  double dt;
};
// e[nj][3] = far-field samples j0 .. j0+nj-1 of Jhist[nsteps][3N] and, if W is
// not null, W[0] = dt sum_j |e_j|^2; partials: scratch of farfield_partials(N, nj) doubles.
size_t farfield_partials(long long N, int nj);
// Largest nj of the allocation-free far field (mot_farfield_static): its
// partials live in a static device array of FF_NJ_MAX * 256 * 3 doubles (6 MiB).
constexpr int FF_NJ_MAX = 1024;
// This device's copy of that array (resolved once per device on first use;
// the calling thread's current device).
hipError_t farfield_scratch(double** p);
hipError_t launch_farfield(const double* Jhist, int nsteps, int nx, int ny, int nz, const FarGeom& g, int j0, int nj,
                           double* partials, double* e, double* W, hipStream_t s);
// g_n[3N] = scale * (transpose of the far field applied to the weights w[nj][3]), step n.
hipError_t launch_farfield_adjoint(const double* w, int j0, int nj, long long n, int nx, int ny, int nz,
                                   const FarGeom& g, double scale, double* g_n, hipStream_t s);
// grad[m] += sum_p lam[p,m] (d_t E^i_p(r_m, t) - w0 J[p,m] - w1 Jprev[p,m] - w2 Jprev2[p,m]
//                            + uh[p,m] + u0[p,m]);  Jprev and Jprev2 may be null (zero).
hipError_t launch_adjoint_grad(const mot_pulse* p, double t, const double* lam, const double* J,
                               const double* Jprev, const double* Jprev2, const double* uh, const double* u0,
                               double* grad, const double* w, int nx, int ny, int nz, hipStream_t s);

}  // namespace motimpl
