// Vector kernels of the device-resident TFQMR (Freund's transpose-free QMR,
// used by the paper for every Z0 solve).  All vectors are FP64.  Inner
// products are deterministic: a fixed grid of RED_BLOCKS blocks writes one
// partial per block (wavefront shuffle, then LDS), and a single block sums
// the partials in a fixed order.  Scalars (rho, alpha, theta, tau, eta, beta)
// live in device memory and are updated by one-thread kernels, so a whole
// iteration is enqueued without a host round trip.
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

__global__ __launch_bounds__(RED_THREADS) void k_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                     long long n, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) acc += a[i] * b[i];
  block_partial(acc, partials);
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce(const double* __restrict__ partials, double* scal,
                                                        int slot, int mode) {
  // one block; each thread sums a fixed strided subset, then fixed tree
  double acc = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += RED_THREADS) {
    const double v = partials[i];
    acc = mode == 0 ? acc + v : fmax(acc, v);
  }
  __shared__ double red[RED_THREADS];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = mode == 0 ? red[threadIdx.x] + red[threadIdx.x + s]
                                                      : fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scal[slot] = red[0];
}

__global__ __launch_bounds__(RED_THREADS) void k_add(const double* __restrict__ a, const double* __restrict__ b,
                                                     double* __restrict__ out, long long n, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double v = a[i] + b[i];
    out[i] = v;
    acc += v * v;
  }
  block_partial(acc, partials);
}

__global__ __launch_bounds__(RED_THREADS) void k_sub(const double* __restrict__ a, const double* __restrict__ b,
                                                     double* __restrict__ out, long long n, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double v = a[i] - b[i];
    out[i] = v;
    acc += v * v;
  }
  block_partial(acc, partials);
}

__global__ void k_copy_scale(const double* __restrict__ a, double alpha, double* __restrict__ out, long long n) {
  GRID_STRIDE(i, n) out[i] = alpha * a[i];
}

__global__ void k_axpy(double* __restrict__ x, const double* __restrict__ d, const double* __restrict__ scal,
                       int slot, long long n) {
  const double e = scal[slot];
  GRID_STRIDE(i, n) x[i] += e * d[i];
}

__global__ void k_zero(double* __restrict__ a, long long n) {
  GRID_STRIDE(i, n) a[i] = 0.0;
}

// w = u = rt = r0, d = 0, x = 0
__global__ void k_tfqmr_init(const double* __restrict__ r0, double* __restrict__ w, double* __restrict__ u,
                             double* __restrict__ rt, double* __restrict__ d, double* __restrict__ x,
                             long long n) {
  GRID_STRIDE(i, n) {
    const double r = r0[i];
    w[i] = r;
    u[i] = r;
    rt[i] = r;
    d[i] = 0.0;
    x[i] = 0.0;
  }
}

// first half step: [x += eta d]; u2 = u - alpha v; w -= alpha au; d = u + dcoef d; |w|^2
__global__ __launch_bounds__(RED_THREADS) void k_half0(double* __restrict__ x, double* __restrict__ u2,
                                                       const double* __restrict__ u, const double* __restrict__ v,
                                                       double* __restrict__ w, const double* __restrict__ au,
                                                       double* __restrict__ d, const double* __restrict__ scal,
                                                       int apply_x, long long n, double* partials) {
  const double alpha = scal[S_ALPHA], dc = scal[S_DCOEF], eta = scal[S_ETA];
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double di = d[i];
    if (apply_x) x[i] += eta * di;
    const double ui = u[i];
    u2[i] = ui - alpha * v[i];
    const double wi = w[i] - alpha * au[i];
    w[i] = wi;
    d[i] = ui + dc * di;
    acc += wi * wi;
  }
  block_partial(acc, partials);
}

// second half step: x += eta d; w -= alpha au2; d = u2 + dcoef d; |w|^2
__global__ __launch_bounds__(RED_THREADS) void k_half1(double* __restrict__ x, double* __restrict__ w,
                                                       const double* __restrict__ au2, double* __restrict__ d,
                                                       const double* __restrict__ u2,
                                                       const double* __restrict__ scal, long long n,
                                                       double* partials) {
  const double alpha = scal[S_ALPHA], dc = scal[S_DCOEF], eta = scal[S_ETA];
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double di = d[i];
    x[i] += eta * di;
    const double wi = w[i] - alpha * au2[i];
    w[i] = wi;
    d[i] = u2[i] + dc * di;
    acc += wi * wi;
  }
  block_partial(acc, partials);
}

// x += eta d (pending update of the second half step); w . rt
__global__ __launch_bounds__(RED_THREADS) void k_rho(double* __restrict__ x, const double* __restrict__ d,
                                                     const double* __restrict__ w, const double* __restrict__ rt,
                                                     const double* __restrict__ scal, long long n,
                                                     double* partials) {
  const double eta = scal[S_ETA];
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    x[i] += eta * d[i];
    acc += w[i] * rt[i];
  }
  block_partial(acc, partials);
}

__global__ void k_u(double* __restrict__ u, const double* __restrict__ w, const double* __restrict__ u2,
                    const double* __restrict__ scal, long long n) {
  const double beta = scal[S_BETA];
  GRID_STRIDE(i, n) u[i] = w[i] + beta * u2[i];
}

// v = au + beta (au2 + beta v); v . rt
__global__ __launch_bounds__(RED_THREADS) void k_v(double* __restrict__ v, const double* __restrict__ au,
                                                   const double* __restrict__ au2, const double* __restrict__ rt,
                                                   const double* __restrict__ scal, long long n,
                                                   double* partials) {
  const double beta = scal[S_BETA];
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double vi = au[i] + beta * (au2[i] + beta * v[i]);
    v[i] = vi;
    acc += vi * rt[i];
  }
  block_partial(acc, partials);
}

// v = au (start); v . rt
__global__ __launch_bounds__(RED_THREADS) void k_v0(double* __restrict__ v, const double* __restrict__ au,
                                                    const double* __restrict__ rt, long long n, double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) {
    const double vi = au[i];
    v[i] = vi;
    acc += vi * rt[i];
  }
  block_partial(acc, partials);
}

// count of non-finite entries
__global__ __launch_bounds__(RED_THREADS) void k_finite(const double* __restrict__ a, long long n,
                                                        double* partials) {
  double acc = 0.0;
  GRID_STRIDE(i, n) acc += isfinite(a[i]) ? 0.0 : 1.0;
  block_partial(acc, partials);
}

// ---- one-thread scalar updates (Freund's recurrences)
// start: rho = |r0|^2 (rt = r0), tau = |r0|, theta = eta = 0
__global__ void k_sc_init(double* scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  scal[S_RHO] = scal[S_B2];
  scal[S_TAU] = sqrt(scal[S_B2]);
  scal[S_THETA] = 0.0;
  scal[S_ETA] = 0.0;
  scal[S_FLAG] = 0.0;
  scal[S_DCOEF] = 0.0;
}

// alpha = rho / sigma; d-coefficient theta^2 eta / alpha of the coming half step
__global__ void k_sc_alpha(double* scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double sigma = scal[S_SIGMA], rho = scal[S_RHO];
  if (sigma == 0.0 || rho == 0.0 || !isfinite(sigma)) {
    scal[S_FLAG] = 1.0;
    scal[S_ALPHA] = 0.0;
    scal[S_DCOEF] = 0.0;
    return;
  }
  const double alpha = rho / sigma;
  scal[S_ALPHA] = alpha;
  scal[S_DCOEF] = scal[S_THETA] * scal[S_THETA] * scal[S_ETA] / alpha;
}

// theta = |w|/tau, c = 1/sqrt(1+theta^2), tau = tau theta c, eta = c^2 alpha
__global__ void k_sc_half(double* scal, int record_tau0) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double alpha = scal[S_ALPHA];
  const double theta = sqrt(scal[S_W2]) / scal[S_TAU];
  const double c = 1.0 / sqrt(1.0 + theta * theta);
  const double tau = scal[S_TAU] * theta * c;
  const double eta = c * c * alpha;
  scal[S_THETA] = theta;
  scal[S_TAU] = tau;
  scal[S_ETA] = eta;
  scal[S_DCOEF] = alpha != 0.0 ? theta * theta * eta / alpha : 0.0;
  if (record_tau0) scal[S_TAU0] = tau;
}

__global__ void k_sc_beta(double* scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double rn = scal[S_RHONEW], rho = scal[S_RHO];
  if (rho == 0.0) {
    scal[S_FLAG] = 1.0;
    scal[S_BETA] = 0.0;
    return;
  }
  scal[S_BETA] = rn / rho;
  scal[S_RHO] = rn;
}

static inline dim3 red_grid() { return dim3(RED_BLOCKS); }
static inline dim3 red_block() { return dim3(RED_THREADS); }

hipError_t dot_partial(const double* a, const double* b, long long n, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, red_grid(), red_block(), 0, s, a, b, n, partials);
  return hipGetLastError();
}
hipError_t reduce_to(const double* partials, double* scal, int slot, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), red_block(), 0, s, partials, scal, slot, mode);
  return hipGetLastError();
}
hipError_t vec_add(const double* a, const double* b, double* out, long long n, double* partials,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_add, red_grid(), red_block(), 0, s, a, b, out, n, partials);
  return hipGetLastError();
}
hipError_t vec_sub(const double* a, const double* b, double* out, long long n, double* partials,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_sub, red_grid(), red_block(), 0, s, a, b, out, n, partials);
  return hipGetLastError();
}
hipError_t vec_copy_scale(const double* a, double alpha, double* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_scale, red_grid(), red_block(), 0, s, a, alpha, out, n);
  return hipGetLastError();
}
hipError_t vec_axpy_inplace(double* x, const double* d, const double* scal, int slot, long long n,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, red_grid(), red_block(), 0, s, x, d, scal, slot, n);
  return hipGetLastError();
}
hipError_t vec_zero(double* a, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, red_grid(), red_block(), 0, s, a, n);
  return hipGetLastError();
}
hipError_t tfqmr_init(const double* r0, double* w, double* u, double* rt, double* d, double* x, long long n,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_tfqmr_init, red_grid(), red_block(), 0, s, r0, w, u, rt, d, x, n);
  return hipGetLastError();
}
hipError_t tfqmr_half0(double* x, double* u2, const double* u, const double* v, double* w, const double* au,
                       double* d, const double* scal, bool apply_x, long long n, double* partials,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_half0, red_grid(), red_block(), 0, s, x, u2, u, v, w, au, d, scal, apply_x ? 1 : 0, n,
                     partials);
  return hipGetLastError();
}
hipError_t tfqmr_half1(double* x, double* w, const double* au2, double* d, const double* u2,
                       const double* scal, long long n, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_half1, red_grid(), red_block(), 0, s, x, w, au2, d, u2, scal, n, partials);
  return hipGetLastError();
}
hipError_t tfqmr_rho(double* x, const double* d, const double* w, const double* rt, const double* scal,
                     long long n, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_rho, red_grid(), red_block(), 0, s, x, d, w, rt, scal, n, partials);
  return hipGetLastError();
}
hipError_t tfqmr_u(double* u, const double* w, const double* u2, const double* scal, long long n,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_u, red_grid(), red_block(), 0, s, u, w, u2, scal, n);
  return hipGetLastError();
}
hipError_t tfqmr_v(double* v, const double* au, const double* au2, const double* rt, const double* scal,
                   long long n, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_v, red_grid(), red_block(), 0, s, v, au, au2, rt, scal, n, partials);
  return hipGetLastError();
}
hipError_t tfqmr_v0(double* v, const double* au, const double* rt, long long n, double* partials,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_v0, red_grid(), red_block(), 0, s, v, au, rt, n, partials);
  return hipGetLastError();
}
hipError_t vec_finite_check(const double* a, long long n, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_finite, red_grid(), red_block(), 0, s, a, n, partials);
  return hipGetLastError();
}
hipError_t sc_init(double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_init, dim3(1), dim3(64), 0, s, scal);
  return hipGetLastError();
}
hipError_t sc_alpha(double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_alpha, dim3(1), dim3(64), 0, s, scal);
  return hipGetLastError();
}
hipError_t sc_half(double* scal, bool record_tau0, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_half, dim3(1), dim3(64), 0, s, scal, record_tau0 ? 1 : 0);
  return hipGetLastError();
}
hipError_t sc_beta(double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_beta, dim3(1), dim3(64), 0, s, scal);
  return hipGetLastError();
}

}  // namespace motimpl
