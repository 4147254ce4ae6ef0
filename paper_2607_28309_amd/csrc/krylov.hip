// Vector kernels of the device-resident TFQMR (Freund's transpose-free QMR,
// used by the paper for every Z0 solve).  Vectors are FP64 or FP32 (the
// inner solve of the refined mode); every inner product accumulates in FP64
// and is deterministic: a fixed grid of RED_BLOCKS blocks writes one partial
// per block (wavefront shuffle, then LDS) and a single block sums the
// partials in a fixed order.  That same block then applies the scalar part
// of Freund's recurrences (alpha, theta, c, tau, eta, beta), so the scalars
// never leave device memory and an iteration needs no host round trip.
#include <hip/hip_runtime.h>

#include "mot_internal.h"

namespace motimpl {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum -> partials[blockIdx.x]; every thread passes its own value.
__device__ __forceinline__ void block_partial(double v, double* partials) {
  __shared__ double red[RED_THREADS / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < RED_THREADS / 64; ++i) t += red[i];
    partials[blockIdx.x] = t;
  }
}

#define GRID_STRIDE(i, n) \
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

template <typename V>
__global__ __launch_bounds__(RED_THREADS) void k_dot(const V* __restrict__ a, const V* __restrict__ b, long long n,
                                                     double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) acc += (double)a[i] * (double)b[i];
  block_partial(acc, partials);
}

// Scalar recurrences applied after a reduction into scal[slot].
__device__ void post_op(double* scal, int post) {
  switch (post) {
    case POST_INIT: {  // rho = |r0|^2 (r~ = r0), tau = |r0|, theta = eta = 0
      const double b2 = scal[S_B2];
      scal[S_RHO] = b2;
      scal[S_TAU] = sqrt(b2);
      scal[S_BNORM] = sqrt(b2);
      scal[S_THETA] = 0.0;
      scal[S_ETA] = 0.0;
      scal[S_FLAG] = 0.0;
      scal[S_DCOEF] = 0.0;
      scal[S_ETAP] = 0.0;
      if (!isfinite(b2)) {  // nothing to iterate on
        scal[S_STATUS] = (double)MOT_ENONFINITE;
        scal[S_DONE] = 1.0;
      } else if (b2 == 0.0) {  // x = 0 after 0 iterations
        scal[S_RELRES] = 0.0;
        scal[S_DONE] = 1.0;
      }
      break;
    }
    case POST_ALPHA: {  // alpha = rho / sigma; d coefficient theta^2 eta / alpha
      const double sigma = scal[S_SIGMA], rho = scal[S_RHO];
      // breakdown: rho or sigma zero, or within the near-breakdown
      // tolerance of zero (relative to |b|^2; 0 by default)
      const double bd = scal[S_BDTOL] * scal[S_B2];
      if (fabs(sigma) <= bd || fabs(rho) <= bd || !isfinite(sigma)) {
        scal[S_FLAG] = 1.0;
        scal[S_ALPHA] = 0.0;
        scal[S_DCOEF] = 0.0;
        break;
      }
      const double alpha = rho / sigma;
      scal[S_ALPHA] = alpha;
      scal[S_DCOEF] = scal[S_THETA] * scal[S_THETA] * scal[S_ETA] / alpha;
      scal[S_NMV] += 1.0;  // the product A u that preceded this reduction
      break;
    }
    case POST_HALF0:
    case POST_HALF1: {  // theta = |w|/tau, c = 1/sqrt(1+theta^2), tau = tau theta c, eta = c^2 alpha
      const double alpha = scal[S_ALPHA];
      const double theta = sqrt(scal[S_W2]) / scal[S_TAU];
      const double c = 1.0 / sqrt(1.0 + theta * theta);
      const double tau = scal[S_TAU] * theta * c;
      const double eta = c * c * alpha;
      scal[S_THETA] = theta;
      scal[S_TAU] = tau;
      scal[S_ETA] = eta;
      scal[S_DCOEF] = alpha != 0.0 ? theta * theta * eta / alpha : 0.0;
      if (post == POST_HALF0) {
        scal[S_TAU0] = tau;
        // a solve ended by the bound may stop after this half step (half
        // step 2 it + 1: bound tau sqrt(2 it + 2)); its x update x += eta d
        // is then the pending one and the product A u2 is not completed
        const double bound = tau * sqrt(2.0 * scal[S_ITER] + 2.0);
        if (scal[S_BOUND_ONLY] != 0.0 && isfinite(bound) && bound <= scal[S_TOL] * scal[S_BNORM]) {
          scal[S_ETAP] = eta;
          scal[S_RELRES] = bound / scal[S_BNORM];
          scal[S_DONE] = 1.0;
        } else {
          scal[S_NMV] += 1.0;  // the product A u2 that follows
        }
      }
      break;
    }
    case POST_BETA: {  // beta = rho'/rho, rho = rho'; end of an iteration: convergence bound
      const double rn = scal[S_RHONEW], rho = scal[S_RHO];
      if (fabs(rho) <= scal[S_BDTOL] * scal[S_B2]) {
        scal[S_FLAG] = 1.0;
        scal[S_BETA] = 0.0;
      } else {
        scal[S_BETA] = rn / rho;
        scal[S_RHO] = rn;
      }
      // the second half step's x update (x += eta d) is applied by the next
      // iteration's first product, or by the residual check
      scal[S_ETAP] = scal[S_ETA];
      const double it = scal[S_ITER] + 1.0;
      scal[S_ITER] = it;
      // quasi-residual bound tau sqrt(2m + 1); its passing, a breakdown or the
      // last iteration ask for the true residual
      const double bound = scal[S_TAU] * sqrt(2.0 * it + 1.0);
      if (!isfinite(bound)) {
        scal[S_STATUS] = (double)MOT_ENONFINITE;
        scal[S_DONE] = 1.0;
      } else if (scal[S_BOUND_ONLY] != 0.0) {
        // the bound decides: converged, broken down or out of iterations
        if (bound <= scal[S_TOL] * scal[S_BNORM]) {
          scal[S_RELRES] = bound / scal[S_BNORM];
          scal[S_DONE] = 1.0;
        } else if (scal[S_FLAG] != 0.0) {
          scal[S_STATUS] = (double)MOT_EBREAKDOWN;
          scal[S_DONE] = 1.0;
        } else if (it >= scal[S_MAXIT]) {
          scal[S_RELRES] = bound / scal[S_BNORM];
          scal[S_STATUS] = (double)MOT_ENOCONV;
          scal[S_DONE] = 1.0;
        }
      } else if (bound <= scal[S_TOL] * scal[S_BNORM] || scal[S_FLAG] != 0.0 || it >= scal[S_MAXIT]) {
        scal[S_CHECK] = 1.0;
      }
      break;
    }
    case POST_RESID: {  // true residual |b - A x|^2 in S_R2 (the check applied the pending x update)
      const double rel = sqrt(scal[S_R2]) / scal[S_BNORM];
      scal[S_RELRES] = rel;
      scal[S_NMV] += 1.0;
      scal[S_ETAP] = 0.0;
      if (!isfinite(rel)) {
        scal[S_STATUS] = (double)MOT_ENONFINITE;
        scal[S_DONE] = 1.0;
      } else if (rel <= scal[S_TOL]) {
        scal[S_DONE] = 1.0;
      } else if (scal[S_FLAG] != 0.0) {
        scal[S_STATUS] = (double)MOT_EBREAKDOWN;
        scal[S_DONE] = 1.0;
      } else if (scal[S_ITER] >= scal[S_MAXIT]) {
        scal[S_STATUS] = (double)MOT_ENOCONV;
        scal[S_DONE] = 1.0;
      } else {
        scal[S_CHECK] = 0.0;
      }
      break;
    }
    default:
      break;
  }
}

// Sum of nparts partials in a fixed order by a block of NT threads (every
// thread returns it).
template <int NT = RED_THREADS>
__device__ __forceinline__ double sum_partials(const double* __restrict__ partials, int nparts) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NT) acc += partials[i];
  __shared__ double red[NT];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// The final sums of the solver's reductions run in one workgroup of
// FIN_THREADS threads: a wide block, so that each thread adds few partials.
constexpr int FIN_THREADS = 1024;

// mirror (optional, host memory the device can write): the scalars are
// copied there after the recurrence, also when the gate is closed, so that
// the host reads the solver's state without a copy command of its own.
__global__ __launch_bounds__(FIN_THREADS) void k_reduce(const double* __restrict__ partials, double* scal,
                                                        int slot, int post, Gate g, int nparts, double* mirror) {
  if (motfft::gate_closed(g)) {
    if (mirror && threadIdx.x < S_NSLOT) mirror[threadIdx.x] = scal[threadIdx.x];
    return;
  }
  const double sum = sum_partials<FIN_THREADS>(partials, nparts);
  if (threadIdx.x == 0) {
    scal[slot] = sum;
    post_op(scal, post);
  }
  if (mirror) {
    __syncthreads();
    if (threadIdx.x < S_NSLOT) mirror[threadIdx.x] = scal[threadIdx.x];
  }
}

// Two sums (partials[0, nparts) and [stride, stride + nparts)), then their
// scalar recurrences in order.
__global__ __launch_bounds__(FIN_THREADS) void k_reduce2(const double* __restrict__ partials, double* scal,
                                                         int slot1, int post1, int slot2, int post2, Gate g,
                                                         int nparts, int stride) {
  if (motfft::gate_closed(g)) return;
  const double s1 = sum_partials<FIN_THREADS>(partials, nparts);
  const double s2 = sum_partials<FIN_THREADS>(partials + stride, nparts);
  if (threadIdx.x == 0) {
    scal[slot1] = s1;
    scal[slot2] = s2;
    post_op(scal, post1);
    post_op(scal, post2);
  }
}

__global__ void k_solver_setup(double* scal, double tol, double max_iter, double bound_only, double bdtol) {
  if (threadIdx.x != 0) return;
  scal[S_BOUND_ONLY] = bound_only;
  scal[S_BDTOL] = bdtol;
  scal[S_TOL] = tol;
  scal[S_MAXIT] = max_iter;
  scal[S_ITER] = 0.0;
  scal[S_DONE] = 0.0;
  scal[S_CHECK] = 0.0;
  scal[S_STATUS] = 0.0;
  scal[S_RELRES] = 0.0;
  scal[S_NMV] = 0.0;
}

template <typename V>
__global__ __launch_bounds__(RED_THREADS) void k_sub(const V* __restrict__ a, const V* __restrict__ b,
                                                     V* __restrict__ out, long long n, double* partials, Gate g) {
  if (motfft::gate_closed(g)) return;
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const V v = a[i] - b[i];
    out[i] = v;
    acc += (double)v * (double)v;
  }
  block_partial(acc, partials);
}

__global__ __launch_bounds__(RED_THREADS) void k_add64(const double* __restrict__ a, const double* __restrict__ b,
                                                       double* __restrict__ out, long long n, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double v = a[i] + b[i];
    out[i] = v;
    acc += v * v;
  }
  block_partial(acc, partials);
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ out, long long n) {
  GRID_STRIDE(i, n) out[i] = a[i];
}

template <typename V>
__global__ void k_zero(V* __restrict__ a, long long n) {
  GRID_STRIDE(i, n) a[i] = (V)0;
}

// Dots of the multidot set: u_j . w_i and u_0 . u_0, partials per dot.
__global__ __launch_bounds__(RED_THREADS) void k_multidot(DotSet ds, long long n, double* partials) {
  constexpr int ND = 2 * PRED_MAX + 1;
  double acc[ND];
#pragma unroll
  for (int q = 0; q < ND; ++q) acc[q] = 0.0;
  GRID_STRIDE(i, n) {
    const double u0 = ds.u[0][i];
    const double u1 = ds.nu > 1 ? ds.u[1][i] : 0.0;
#pragma unroll
    for (int k = 0; k < PRED_MAX; ++k)
      if (k < ds.nw) {
        const double w = ds.w[k][i];
        acc[k] += u0 * w;
        acc[PRED_MAX + k] += u1 * w;
      }
    acc[2 * PRED_MAX] += u0 * u0;
  }
  // partials of dot (j, k) at (j nw + k) RED_BLOCKS; the self dot after them
#pragma unroll
  for (int q = 0; q < ND; ++q) {
    const int j = q / PRED_MAX, k = q % PRED_MAX;
    const bool used = q == 2 * PRED_MAX || (j < ds.nu && k < ds.nw);
    const int slot = q == 2 * PRED_MAX ? ds.nu * ds.nw : j * ds.nw + k;
    if (used) block_partial(acc[q], partials + (size_t)slot * RED_BLOCKS);
    __syncthreads();  // block_partial's LDS is reused by the next dot
  }
}

// out[d] = sum of partials[d RED_BLOCKS ...] (one block per dot)
__global__ __launch_bounds__(RED_THREADS) void k_reduce_many(const double* __restrict__ partials, double* out) {
  const double sum = sum_partials(partials + (size_t)blockIdx.x * RED_BLOCKS, RED_BLOCKS);
  if (threadIdx.x == 0) out[blockIdx.x] = sum;
}

__global__ void k_pred_combine(Combo cb, const double* __restrict__ b, double* __restrict__ x0,
                               double* __restrict__ r0, long long n) {
  GRID_STRIDE(i, n) {
    double x = 0.0, z = 0.0;
#pragma unroll
    for (int k = 0; k < PRED_MAX; ++k)
      if (k < cb.k) {
        x += cb.c[k] * cb.J[k][i];
        z += cb.c[k] * cb.Z[k][i];
      }
    x0[i] = x;
    r0[i] = b[i] - z;
  }
}

// x *= rs (per voxel: x holds three components of nvox values each)
template <typename V>
__global__ void k_scale_voxel(V* __restrict__ x, const V* __restrict__ rs, long long n, long long nvox) {
  GRID_STRIDE(i, n) x[i] *= rs[i % nvox];
}

// The end of an inner FP32 solve handed to the FP64 iterate: per voxel v and
// component, t = (x32 + coef d) rs[v] in FP32 (coef null: no update), then
// x64 = t or x64 += t.
__global__ void k_finish_f2d(const float* __restrict__ x32, const float* __restrict__ d,
                             const double* __restrict__ coef, const float* __restrict__ rs,
                             double* __restrict__ x64, long long nvox, int acc) {
  const float a = coef ? (float)*coef : 0.0f;
  GRID_STRIDE(v, nvox) {
    const float r = rs[v];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long i = c * nvox + v;
      float t = x32[i];
      if (coef) t += a * d[i];
      t *= r;
      x64[i] = acc ? x64[i] + (double)t : (double)t;
    }
  }
}

// x += coef d (coef read on the device)
template <typename V>
__global__ void k_axpy_scal(V* __restrict__ x, const V* __restrict__ d, const double* __restrict__ coef,
                            long long n) {
  const V a = (V)*coef;
  GRID_STRIDE(i, n) x[i] += a * d[i];
}

// w = u = rt = r0, d = 0, x = 0
template <typename V>
__global__ void k_tfqmr_init(const V* __restrict__ r0, V* __restrict__ w, V* __restrict__ u, V* __restrict__ rt,
                             V* __restrict__ d, V* __restrict__ x, long long n) {
  GRID_STRIDE(i, n) {
    const V r = r0[i];
    w[i] = r;
    u[i] = r;
    rt[i] = r;
    d[i] = (V)0;
    x[i] = (V)0;
  }
}

// w = u = rt = (float) r0, d = 0, x = 0, and |w|^2 partials (the start of
// an inner FP32 solve on an FP64 residual)
__global__ __launch_bounds__(RED_THREADS) void k_tfqmr_init_d2f(const double* __restrict__ r0, float* __restrict__ w,
                                                                float* __restrict__ u, float* __restrict__ rt,
                                                                float* __restrict__ d, float* __restrict__ x,
                                                                long long n, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const float r = (float)r0[i];
    w[i] = r;
    u[i] = r;
    rt[i] = r;
    d[i] = 0.0f;
    x[i] = 0.0f;
    acc += (double)r * (double)r;
  }
  block_partial(acc, partials);
}

// v = au (start); v . rt
template <typename V>
__global__ __launch_bounds__(RED_THREADS) void k_v0(V* __restrict__ v, const V* __restrict__ au,
                                                    const V* __restrict__ rt, long long n, double* partials, Gate g) {
  if (motfft::gate_closed(g)) return;
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const V vi = au[i];
    v[i] = vi;
    acc += (double)vi * (double)rt[i];
  }
  block_partial(acc, partials);
}

static inline dim3 RG() { return dim3(RED_BLOCKS); }
static inline dim3 RB() { return dim3(RED_THREADS); }
#define LAUNCH(kernel, ...)                                        \
  do {                                                             \
    hipLaunchKernelGGL(kernel, RG(), RB(), 0, s, __VA_ARGS__);     \
    return hipGetLastError();                                      \
  } while (0)

template <typename V>
hipError_t dot_partial(const V* a, const V* b, long long n, double* partials, hipStream_t s) {
  LAUNCH(k_dot<V>, a, b, n, partials);
}
hipError_t reduce_post(const double* partials, double* scal, int slot, int post, hipStream_t s, Gate g,
                       int nparts, double* mirror) {
  if (nparts < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(FIN_THREADS), 0, s, partials, scal, slot, post, g, nparts, mirror);
  return hipGetLastError();
}
hipError_t reduce_post2(const double* partials, double* scal, int slot1, int post1, int slot2, int post2,
                        hipStream_t s, Gate g, int nparts, int stride) {
  if (nparts < 1 || stride < nparts) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(FIN_THREADS), 0, s, partials, scal, slot1, post1, slot2, post2, g,
                     nparts, stride);
  return hipGetLastError();
}
hipError_t solver_setup(double* scal, double tol, int max_iter, hipStream_t s, bool bound_only, double breakdown_tol) {
  hipLaunchKernelGGL(k_solver_setup, dim3(1), dim3(64), 0, s, scal, tol, (double)max_iter, bound_only ? 1.0 : 0.0,
                     breakdown_tol);
  return hipGetLastError();
}
template <typename V>
hipError_t vec_axpy_scal(V* x, const V* d, const double* coef, long long n, hipStream_t s) {
  LAUNCH(k_axpy_scal<V>, x, d, coef, n);
}
template <typename V>
hipError_t vec_scale_voxel(V* x, const V* rs, long long n, long long nvox, hipStream_t s) {
  LAUNCH(k_scale_voxel<V>, x, rs, n, nvox);
}
hipError_t finish_f2d(const float* x32, const float* d, const double* coef, const float* rs, double* x64,
                      long long nvox, bool acc, hipStream_t s) {
  LAUNCH(k_finish_f2d, x32, d, coef, rs, x64, nvox, acc ? 1 : 0);
}
hipError_t multidot(const DotSet& ds, long long n, double* partials, double* out, hipStream_t s) {
  if (ds.nu < 1 || ds.nu > 2 || ds.nw < 0 || ds.nw > PRED_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_multidot, RG(), RB(), 0, s, ds, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_many, dim3(ds.nu * ds.nw + 1), RB(), 0, s, partials, out);
  return hipGetLastError();
}
hipError_t pred_combine(const Combo& cb, const double* b, double* x0, double* r0, long long n, hipStream_t s) {
  if (cb.k < 1 || cb.k > PRED_MAX) return hipErrorInvalidValue;
  LAUNCH(k_pred_combine, cb, b, x0, r0, n);
}
template <typename V>
hipError_t vec_sub(const V* a, const V* b, V* out, long long n, double* partials, hipStream_t s, Gate g) {
  LAUNCH(k_sub<V>, a, b, out, n, partials, g);
}
hipError_t vec_add64(const double* a, const double* b, double* out, long long n, double* partials, hipStream_t s) {
  LAUNCH(k_add64, a, b, out, n, partials);
}
hipError_t vec_copy(const double* a, double* out, long long n, hipStream_t s) { LAUNCH(k_copy, a, out, n); }
template <typename V>
hipError_t vec_zero(V* a, long long n, hipStream_t s) {
  LAUNCH(k_zero<V>, a, n);
}
template <typename V>
hipError_t tfqmr_init(const V* r0, V* w, V* u, V* rt, V* d, V* x, long long n, hipStream_t s) {
  LAUNCH(k_tfqmr_init<V>, r0, w, u, rt, d, x, n);
}
hipError_t tfqmr_init_d2f(const double* r0, float* w, float* u, float* rt, float* d, float* x, long long n,
                          double* partials, hipStream_t s) {
  LAUNCH(k_tfqmr_init_d2f, r0, w, u, rt, d, x, n, partials);
}
template <typename V>
hipError_t tfqmr_v0(V* v, const V* au, const V* rt, long long n, double* partials, hipStream_t s, Gate g) {
  LAUNCH(k_v0<V>, v, au, rt, n, partials, g);
}

#define INST(V)                                                                                              \
  template hipError_t dot_partial<V>(const V*, const V*, long long, double*, hipStream_t);                    \
  template hipError_t vec_sub<V>(const V*, const V*, V*, long long, double*, hipStream_t, Gate);              \
  template hipError_t vec_zero<V>(V*, long long, hipStream_t);                                                \
  template hipError_t tfqmr_init<V>(const V*, V*, V*, V*, V*, V*, long long, hipStream_t);                    \
  template hipError_t vec_axpy_scal<V>(V*, const V*, const double*, long long, hipStream_t);                  \
  template hipError_t vec_scale_voxel<V>(V*, const V*, long long, long long, hipStream_t);                   \
  template hipError_t tfqmr_v0<V>(V*, const V*, const V*, long long, double*, hipStream_t, Gate);
INST(float)
INST(double)
#undef INST

}  // namespace motimpl
