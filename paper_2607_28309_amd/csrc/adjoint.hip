// Far-field signature of a current history, its transpose and the
// permittivity gradient of the adjoint march.
//
// The current J(r_m, t) = sum_n J_{m,n} T(t/dt - n) (the basis of Sec. II)
// radiates through the retarded vector potential of Eq. 1; far away in the
// unit direction r (common factor 1/(4 pi R) and delay R dropped, c0 = mu0 =
// h = 1) its field sampled at tau_j = j dt is
//   e_j = -(1/(4 pi dt)) P sum_m sum_n J_{m,n} T'(j - n + s_m),
// with s_m = r . r_m / dt, r_m the voxel centre relative to the grid centre,
// P = I - r r^T and T' the spline derivative in step units.  The transpose
// maps weights w_j to g_n(m) = -(1/(4 pi dt)) sum_j T'(j - n + s_m) P w_j.
//
// Gradient of W(eps) through the adjoint currents lam_n (the transposed
// march, Z_k^T = T(k) diag(eps) - G_k diag(eps - 1)):
//   dW/d eps_m = sum_n lam_n(m) . (d_t E^i(r_m, t_n) - sum_k w_k J_{n-k}(m) + u_n(m)),
// w = (1/2, 1/2, 0) plus the regularization's (d_0, d_1, d_2),
// u_n = sum_k G_k J_{n-k} (given as its history and present parts): the derivative of the excitation (Eq. 7) and of
// the diagonal and contrast parts of every Z_k with respect to eps_m.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mot_internal.h"

namespace motimpl {

namespace {

constexpr int FF_THREADS = 256;
constexpr int FF_BLOCKS = 256;  // fixed partial count per sample: deterministic sums

// Far-field partials of the allocation-free entry point: one copy per GPU,
// held until the process ends.  Host code never uses this name as an
// address: it resolves each device's copy with hipGetSymbolAddress once
// (farfield_scratch) and passes that pointer to the kernels.
constexpr size_t FF_SCRATCH_DOUBLES = (size_t)FF_NJ_MAX * FF_BLOCKS * 3;
static __device__ __align__(256) double scratch[FF_SCRATCH_DOUBLES];

constexpr int FF_MAX_DEVICES = 64;
std::once_flag scratch_once[FF_MAX_DEVICES];
double* scratch_ptr[FF_MAX_DEVICES];
hipError_t scratch_err[FF_MAX_DEVICES];

__device__ __forceinline__ double dspline(double s) {
  if (s >= -1.0 && s < 0.0) return s + 1.0;
  if (s >= 0.0 && s < 1.0) return 1.0 - 2.0 * s;
  if (s >= 1.0 && s < 2.0) return s - 2.0;
  return 0.0;
}

__device__ __forceinline__ double shift(const FarGeom& g, long long m, int nx, int ny, int nz) {
  double x, y, z;
  voxel_centre(m, nx, ny, nz, x, y, z);
  return (g.r[0] * x + g.r[1] * y + g.r[2] * z) / g.dt;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < FF_THREADS / 64; ++i) t += red[i];
  return t;
}

// partials[(jj * FF_BLOCKS + b) * 3 + p]: block b's share of sample j0 + jj
__global__ __launch_bounds__(FF_THREADS) void k_farfield_part(const double* __restrict__ Jh, int nsteps, int nx,
                                                              int ny, int nz, FarGeom g, int j0,
                                                              double* __restrict__ part) {
  __shared__ double red[FF_THREADS / 64];
  const long long N = (long long)nx * ny * nz;
  const int jj = blockIdx.y;
  const double j = (double)(j0 + jj);
  double a[3] = {0.0, 0.0, 0.0};
  for (long long m = (long long)blockIdx.x * FF_THREADS + threadIdx.x; m < N; m += (long long)FF_BLOCKS * FF_THREADS) {
    const double s = shift(g, m, nx, ny, nz);
    // T'(j - n + s) vanishes unless j + s - 2 < n <= j + s + 1
    int nlo = (int)floor(j + s - 2.0), nhi = (int)floor(j + s + 1.0);
    nlo = nlo < 0 ? 0 : nlo;
    nhi = nhi > nsteps - 1 ? nsteps - 1 : nhi;
    for (int n = nlo; n <= nhi; ++n) {
      const double w = dspline((double)(j0 + jj - n) + s);
      if (w == 0.0) continue;
      const double* Jn = Jh + (size_t)n * 3 * N;
#pragma unroll
      for (int p = 0; p < 3; ++p) a[p] += w * Jn[p * N + m];
    }
  }
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const double t = block_sum(a[p], red);
    if (threadIdx.x == 0) part[((size_t)jj * FF_BLOCKS + blockIdx.x) * 3 + p] = t;
  }
}

__global__ void k_farfield_final(const double* __restrict__ part, int nj, FarGeom g, double* __restrict__ e) {
  const int jj = blockIdx.x * blockDim.x + threadIdx.x;
  if (jj >= nj) return;
  double a[3] = {0.0, 0.0, 0.0};
  for (int b = 0; b < FF_BLOCKS; ++b)
#pragma unroll
    for (int p = 0; p < 3; ++p) a[p] += part[((size_t)jj * FF_BLOCKS + b) * 3 + p];
  const double sc = -1.0 / (4.0 * 3.14159265358979323846 * g.dt);
#pragma unroll
  for (int p = 0; p < 3; ++p) e[jj * 3 + p] = sc * (g.P[3 * p] * a[0] + g.P[3 * p + 1] * a[1] + g.P[3 * p + 2] * a[2]);
}

// W = dt sum_j |e_j|^2 in one block, fixed order
__global__ __launch_bounds__(FF_THREADS) void k_farfield_energy(const double* __restrict__ e, int nj, double dt,
                                                                double* __restrict__ W) {
  __shared__ double red[FF_THREADS / 64];
  double a = 0.0;
  for (int i = threadIdx.x; i < 3 * nj; i += FF_THREADS) a += e[i] * e[i];
  const double t = block_sum(a, red);
  if (threadIdx.x == 0) W[0] = dt * t;
}

__global__ void k_farfield_adj(const double* __restrict__ w, int j0, int nj, long long n, int nx, int ny, int nz,
                               FarGeom g, double scale, double* __restrict__ out) {
  const long long N = (long long)nx * ny * nz;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const double s = shift(g, m, nx, ny, nz);
  // T'(j - n + s) vanishes unless n - s - 1 <= j < n - s + 2
  int jlo = (int)floor((double)n - s - 1.0), jhi = (int)floor((double)n - s + 2.0);
  jlo = jlo < j0 ? j0 : jlo;
  jhi = jhi > j0 + nj - 1 ? j0 + nj - 1 : jhi;
  double a[3] = {0.0, 0.0, 0.0};
  for (int j = jlo; j <= jhi; ++j) {
    const double t = dspline((double)(j - n) + s);
    if (t == 0.0) continue;
    const double* wj = w + (size_t)(j - j0) * 3;
#pragma unroll
    for (int p = 0; p < 3; ++p) a[p] += t * (g.P[3 * p] * wj[0] + g.P[3 * p + 1] * wj[1] + g.P[3 * p + 2] * wj[2]);
  }
  const double sc = -scale / (4.0 * 3.14159265358979323846 * g.dt);
#pragma unroll
  for (int p = 0; p < 3; ++p) out[p * N + m] = sc * a[p];
}

__global__ void k_adjoint_grad(mot_pulse pl, double t, const double* __restrict__ lam, const double* __restrict__ J,
                               const double* __restrict__ Jprev, const double* __restrict__ Jprev2,
                               const double* __restrict__ uh, const double* __restrict__ u0,
                               double* __restrict__ grad, double w0, double w1, double w2, int nx, int ny, int nz) {
  const long long N = (long long)nx * ny * nz;
  const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  double x, y, z;
  voxel_centre(m, nx, ny, nz, x, y, z);
  const double di = incident_dt(pl, t, x, y, z);
  double acc = 0.0;
#pragma unroll
  for (int p = 0; p < 3; ++p) {
    const long long i = p * N + m;
    double jj = w0 * J[i];
    if (Jprev) jj += w1 * Jprev[i];
    if (Jprev2) jj += w2 * Jprev2[i];
    acc += lam[i] * (di * pl.e[p] - jj + (uh[i] + u0[i]));
  }
  grad[m] += acc;
}

}  // namespace

size_t farfield_partials(long long, int nj) { return (size_t)nj * FF_BLOCKS * 3; }

hipError_t farfield_scratch(double** p) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= FF_MAX_DEVICES) return hipErrorInvalidDevice;
  // once per device, with that device current (it is the caller's current one)
  std::call_once(scratch_once[dev], [dev] {
    void* q = nullptr;
    scratch_err[dev] = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    scratch_ptr[dev] = scratch_err[dev] == hipSuccess ? (double*)q : nullptr;
  });
  if (scratch_err[dev] != hipSuccess) return scratch_err[dev];
  *p = scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_farfield(const double* Jhist, int nsteps, int nx, int ny, int nz, const FarGeom& g, int j0, int nj,
                           double* partials, double* e, double* W, hipStream_t s) {
  hipLaunchKernelGGL(k_farfield_part, dim3(FF_BLOCKS, nj), dim3(FF_THREADS), 0, s, Jhist, nsteps, nx, ny, nz, g, j0,
                     partials);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_farfield_final, dim3((nj + 63) / 64), dim3(64), 0, s, partials, nj, g, e);
  err = hipGetLastError();
  if (err != hipSuccess || !W) return err;
  hipLaunchKernelGGL(k_farfield_energy, dim3(1), dim3(FF_THREADS), 0, s, e, nj, g.dt, W);
  return hipGetLastError();
}

hipError_t launch_farfield_adjoint(const double* w, int j0, int nj, long long n, int nx, int ny, int nz,
                                   const FarGeom& g, double scale, double* g_n, hipStream_t s) {
  const long long N = (long long)nx * ny * nz;
  hipLaunchKernelGGL(k_farfield_adj, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, w, j0, nj, n, nx, ny, nz, g,
                     scale, g_n);
  return hipGetLastError();
}

hipError_t launch_adjoint_grad(const mot_pulse* p, double t, const double* lam, const double* J,
                               const double* Jprev, const double* Jprev2, const double* uh, const double* u0,
                               double* grad, const double* w, int nx, int ny, int nz, hipStream_t s) {
  const long long N = (long long)nx * ny * nz;
  hipLaunchKernelGGL(k_adjoint_grad, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, *p, t, lam, J, Jprev,
                     Jprev2, uh, u0, grad, w[0], w[1], w[2], nx, ny, nz);
  return hipGetLastError();
}

}  // namespace motimpl
