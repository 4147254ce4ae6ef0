// Retarded Green dyad G_k(d) of the voxel discretization, its circulant
// embedding and the real spectra Lambda_k (Sec. IV, Eq. 10 and Eq. 11).
//
// G_k(d)[p,q] = d_p d_q Pi_k - delta_pq d_t^2 Pi_k + delta_pq T(k)[d=0], with
// Pi_k(d) = int over the source box B(d) of T(k - R/L)/(4 pi R) (observation
// at a voxel centre, units c0 = h = 1, L = c0 dt/h, T the causal quadratic
// spline with T(0) = T(1) = 1/2).  By the divergence theorem:
//   off-diagonal  A_pq = sum_{sp,sq} sp sq int f(R) dx_r over the four box
//                 edges parallel to the third axis, f(R) = T(k-R/L)/(4 pi R);
//   diagonal      A_pp = sum_s s a_s iint_{x_p = a_s} f'(R)/R dS;
//   time term     B = -sum_faces (n.x') iint H(R)/R^3 dS,
//                 H(R) = (1/(4 pi L^2)) int_0^R T''(k - r/L) r dr.
// A face integral of a radial function phi with phi(R) R = Phi'(R) is taken
// in polar form about the foot of the observation point on the face plane:
//   iint phi dS = sum over the four edges of int Phi(R) dtheta
//                 - 2 pi Phi(|a|) [foot inside the face],
// where along an edge at in-plane offset h, dtheta = h ds/(h^2 + s^2).  Every
// 1-D integrand is smooth between the points where R crosses a knot sphere
// R = (k-2)L, ..., (k+1)L; those points split the edges, and each piece is
// integrated by Gauss-Legendre.  Phi = f for A_pp, Phi = K (K' = H/R^2) for B.
#include <hip/hip_runtime.h>

#include "fft_passes.h"
#include "mot_internal.h"

namespace motgreen {

constexpr double PI = 3.14159265358979323846;
constexpr double FOUR_PI = 4.0 * PI;
constexpr int MAXQ = 32;

struct Rule {
  double x[MAXQ];  // nodes on [-1, 1]
  double w[MAXQ];
  int n;
};

// causal quadratic spline, step units
__device__ __forceinline__ double spline(double s) {
  if (s < -1.0 || s >= 2.0) return 0.0;
  if (s < 0.0) return 0.5 * (s + 1.0) * (s + 1.0);
  if (s < 1.0) return 0.75 - (s - 0.5) * (s - 0.5);
  return 0.5 * (2.0 - s) * (2.0 - s);
}

__device__ __forceinline__ double f_rad(double R, double k, double L) {
  return spline(k - R / L) / (FOUR_PI * R);
}

// K(R) = int_0^R H(r)/r^2 dr, H = Q/(4 pi L^2), Q(r) = int_0^r T''(k - u/L) u du.
// T'' (in step units) is +1, -2, +1 on the radial intervals
// [(k-2)L,(k-1)L], [(k-1)L,kL], [kL,(k+1)L] (clipped at 0).
__device__ double k_rad(double R, double k, double L) {
  const double rb[4] = {fmax((k - 2.0) * L, 0.0), fmax((k - 1.0) * L, 0.0), fmax(k * L, 0.0), (k + 1.0) * L};
  const double cs[3] = {1.0, -2.0, 1.0};
  double Q = 0.0, Kv = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double lo = rb[i], hi = rb[i + 1];
    if (hi <= lo) continue;
    if (R <= lo) return Kv / (FOUR_PI * L * L);
    const double top = fmin(R, hi);
    const double E = Q - cs[i] * lo * lo * 0.5;
    Kv += cs[i] * (top - lo) * 0.5;
    if (lo > 0.0) Kv += E * (1.0 / lo - 1.0 / top);
    Q += cs[i] * (top * top - lo * lo) * 0.5;
    if (R <= hi) return Kv / (FOUR_PI * L * L);
  }
  Kv += Q * (1.0 / rb[3] - 1.0 / R);
  return Kv / (FOUR_PI * L * L);
}

// Sorted split points of [s0, s1] where a^2 + h^2 + s^2 crosses a knot radius.
__device__ __forceinline__ int splits(double c2, double s0, double s1, double k, double L, double* pts) {
  int n = 0;
  pts[n++] = s0;
  for (int j = -2; j <= 1; ++j) {
    const double Rk = (k + j) * L;
    if (Rk <= 0.0) continue;
    const double d2 = Rk * Rk - c2;
    if (d2 <= 0.0) continue;
    const double s = sqrt(d2);
    if (-s > s0 && -s < s1) pts[n++] = -s;
    if (s > s0 && s < s1) pts[n++] = s;
  }
  pts[n++] = s1;
  for (int i = 1; i < n; ++i) {  // insertion sort, n <= 10
    double v = pts[i];
    int j = i - 1;
    while (j >= 0 && pts[j] > v) {
      pts[j + 1] = pts[j];
      --j;
    }
    pts[j + 1] = v;
  }
  return n;
}

// int_{s0}^{s1} Phi(sqrt(a^2+h^2+s^2)) h/(h^2+s^2) ds, Phi = f (which==0) or K.
__device__ double edge_angle(int which, double a, double h, double s0, double s1, double k, double L,
                             const Rule& q) {
  double pts[10];
  const double c2 = a * a + h * h;
  const int n = splits(c2, s0, s1, k, L, pts);
  double tot = 0.0;
  for (int i = 0; i + 1 < n; ++i) {
    const double mid = 0.5 * (pts[i] + pts[i + 1]), hw = 0.5 * (pts[i + 1] - pts[i]);
    if (hw <= 0.0) continue;
    double acc = 0.0;
    for (int t = 0; t < q.n; ++t) {
      const double s = mid + hw * q.x[t];
      const double R = sqrt(c2 + s * s);
      const double phi = which == 0 ? f_rad(R, k, L) : k_rad(R, k, L);
      acc += q.w[t] * phi * h / (h * h + s * s);
    }
    tot += hw * acc;
  }
  return tot;
}

// iint over the face [u0,u1]x[v0,v1] in the plane at height a of phi, Phi' = phi R.
__device__ double face_polar(int which, double a, double u0, double u1, double v0, double v1, double k,
                             double L, const Rule& q) {
  double I = edge_angle(which, a, u1, v0, v1, k, L, q) - edge_angle(which, a, u0, v0, v1, k, L, q) +
             edge_angle(which, a, v1, u0, u1, k, L, q) - edge_angle(which, a, v0, u0, u1, k, L, q);
  if (u0 < 0.0 && u1 > 0.0 && v0 < 0.0 && v1 > 0.0) {
    const double ra = fabs(a);
    I -= 2.0 * PI * (which == 0 ? f_rad(ra, k, L) : k_rad(ra, k, L));
  }
  return I;
}

// int_{z0}^{z1} f(sqrt(rho2 + z^2)) dz
__device__ double edge_plain(double rho2, double z0, double z1, double k, double L, const Rule& q) {
  double pts[10];
  const int n = splits(rho2, z0, z1, k, L, pts);
  double tot = 0.0;
  for (int i = 0; i + 1 < n; ++i) {
    const double mid = 0.5 * (pts[i] + pts[i + 1]), hw = 0.5 * (pts[i + 1] - pts[i]);
    if (hw <= 0.0) continue;
    double acc = 0.0;
    for (int t = 0; t < q.n; ++t) {
      const double z = mid + hw * q.x[t];
      acc += q.w[t] * f_rad(sqrt(rho2 + z * z), k, L);
    }
    tot += hw * acc;
  }
  return tot;
}

// Causal-region test M_k(d) (integer-exact for integer alpha).
__device__ __forceinline__ bool in_mask(int ax, int ay, int az, int k, int alpha, double L) {
  if (alpha > 0) {
    const long long a2 = (long long)alpha * alpha;
    auto m1 = [](int v) { return (long long)(v > 0 ? 2 * v - 1 : 0); };
    const long long lo = 3 * (m1(ax) * m1(ax) + m1(ay) * m1(ay) + m1(az) * m1(az));
    if (!(lo < 4LL * (k + 1) * (k + 1) * a2)) return false;
    if (k <= 2) return true;
    const long long hi = 3LL * ((2LL * ax + 1) * (2LL * ax + 1) + (2LL * ay + 1) * (2LL * ay + 1) +
                               (2LL * az + 1) * (2LL * az + 1));
    return hi > 4LL * (k - 2) * (k - 2) * a2;
  }
  const double mx = fmax(ax - 0.5, 0.0), my = fmax(ay - 0.5, 0.0), mz = fmax(az - 0.5, 0.0);
  const double dmin = sqrt(mx * mx + my * my + mz * mz);
  const double dmax = sqrt((ax + 0.5) * (ax + 0.5) + (ay + 0.5) * (ay + 0.5) + (az + 0.5) * (az + 0.5));
  return dmin < (k + 1) * L && dmax > (k - 2) * L;
}

// One thread per non-negative offset d; out[c][dz][dy][dx], c in (xx,yy,zz,xy,xz,yz).
__global__ __launch_bounds__(128) void k_green(double* __restrict__ out, int nx, int ny, int nz, int k,
                                               int alpha, double L, Rule q) {
  const long long N = (long long)nx * ny * nz;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N) return;
  const int ix = (int)(id % nx), iy = (int)((id / nx) % ny), iz = (int)(id / ((long long)nx * ny));
  double g[6] = {0, 0, 0, 0, 0, 0};
  if (in_mask(ix, iy, iz, k, alpha, L)) {
    const double d[3] = {(double)ix, (double)iy, (double)iz};
    const double kk = (double)k;
    double B = 0.0;
    for (int p = 0; p < 3; ++p) {
      const int q1 = p == 0 ? 1 : 0, q2 = p == 2 ? 1 : 2;
      for (int sg = -1; sg <= 1; sg += 2) {
        const double a = d[p] + 0.5 * sg;
        const double u0 = d[q1] - 0.5, u1 = d[q1] + 0.5, v0 = d[q2] - 0.5, v1 = d[q2] + 0.5;
        g[p] += sg * a * face_polar(0, a, u0, u1, v0, v1, kk, L, q);
        B -= sg * a * face_polar(1, a, u0, u1, v0, v1, kk, L, q);
      }
    }
    const double tk = (ix == 0 && iy == 0 && iz == 0) ? spline(kk) : 0.0;
    for (int p = 0; p < 3; ++p) g[p] += B + tk;
    const int pp[3] = {0, 0, 1}, qq[3] = {1, 2, 2};
    for (int c = 0; c < 3; ++c) {
      const int p = pp[c], qd = qq[c], r = 3 - p - qd;
      if (d[p] == 0.0 || d[qd] == 0.0) continue;
      double acc = 0.0;
      for (int sp = -1; sp <= 1; sp += 2)
        for (int sq = -1; sq <= 1; sq += 2) {
          const double xp = d[p] + 0.5 * sp, xq = d[qd] + 0.5 * sq;
          acc += sp * sq * edge_plain(xp * xp + xq * xq, d[r] - 0.5, d[r] + 0.5, kk, L, q);
        }
      g[3 + c] = acc;
    }
  }
  for (int c = 0; c < 6; ++c) out[c * N + id] = g[c];
}

// Circulant embedding of one component on the doubled grid P = 2N:
// index i <-> offset i (i < N), none (i = N), i - P (i > N).
__global__ void k_embed(const double* __restrict__ goct, double* __restrict__ E, int comp, int nx, int ny,
                        int nz) {
  const int px = 2 * nx, py = 2 * ny, pz = 2 * nz;
  const long long tot = (long long)px * py * pz;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= tot) return;
  const int x = (int)(id % px), y = (int)((id / px) % py), z = (int)(id / ((long long)px * py));
  double v = 0.0;
  if (x != nx && y != ny && z != nz) {
    const int ax = x < nx ? x : px - x, ay = y < ny ? y : py - y, az = z < nz ? z : pz - z;
    const int sx = x < nx ? 1 : -1, sy = y < ny ? 1 : -1, sz = z < nz ? 1 : -1;
    const long long N = (long long)nx * ny * nz;
    v = goct[comp * N + ((long long)az * ny + ay) * nx + ax];
    // odd-odd components change sign under reflection of either of their axes
    if (comp == 3) v *= sx * sy;
    if (comp == 4) v *= sx * sz;
    if (comp == 5) v *= sy * sz;
  }
  E[id] = v;
}

// Octant compression of the real spectrum, scaled by 1/(Px Py Pz), for
// kx <= Nx, kyc <= Ny, kzc <= Nz: layout [comp][kzc][kyc][kxs] (tile = 0, read
// by the history multiply-accumulate) or [kyc][kx][kzc][comp] (tile = 1, read
// by the fused z pass, one contiguous range per kx tile).  The largest
// |imaginary part| of each block goes to imax[block] (the embedded kernels
// are even or odd-odd per axis, so the spectra are real up to rounding).
__global__ void k_compress(const double2* __restrict__ spec, double* __restrict__ lam64,
                           float* __restrict__ lam32, double* __restrict__ imax, int comp, int nx, int ny,
                           int nz, int kxs, double scale, int w64, int w32) {
  const int py = 2 * ny;
  const long long cnt = (long long)(nx + 1) * (ny + 1) * (nz + 1);
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double im = 0.0;
  if (id < cnt) {
    const int kx = (int)(id % (nx + 1)), ky = (int)((id / (nx + 1)) % (ny + 1)),
              kz = (int)(id / ((long long)(nx + 1) * (ny + 1)));
    const double2 v = spec[((long long)kz * py + ky) * kxs + kx];
    // w > 0: tile layout of the fused z pass; w = 0: [comp][kz][ky][kxs]
    const size_t plain = (((size_t)comp * (nz + 1) + kz) * (ny + 1) + ky) * kxs + kx;
    const double r = v.x * scale;
    if (lam64) lam64[w64 ? motfft::lam_tile_offset(kx, ky, kz, comp, nx + 1, nz + 1, w64) : plain] = r;
    if (lam32) lam32[w32 ? motfft::lam_tile_offset(kx, ky, kz, comp, nx + 1, nz + 1, w32) : plain] = (float)r;
    im = fabs(v.y) * scale;
  }
  __shared__ double red[256];
  red[threadIdx.x] = im;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) imax[blockIdx.x] = red[0];
}

}  // namespace motgreen

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on P_n, FP64).
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = cos(motgreen::PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
      }
      const double dp = n * (z * p0 - p1) / (z * z - 1.0);
      const double dz = p0 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) {
        // final derivative at the converged node
        double q0 = 1.0, q1 = 0.0;
        for (int j = 1; j <= n; ++j) {
          double q2 = q1;
          q1 = q0;
          q0 = ((2.0 * j - 1.0) * z * q1 - (j - 1.0) * q2) / j;
        }
        const double d = n * (z * q0 - q1) / (z * z - 1.0);
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * d * d);
        break;
      }
    }
  }
}

namespace motimpl {

hipError_t launch_green(double* out, int nx, int ny, int nz, int k, int alpha, double L, int nq,
                        hipStream_t s) {
  motgreen::Rule q;
  if (nq < 2 || nq > motgreen::MAXQ) return hipErrorInvalidValue;
  q.n = nq;
  gauss_legendre(nq, q.x, q.w);
  const long long N = (long long)nx * ny * nz;
  hipLaunchKernelGGL(motgreen::k_green, dim3((unsigned)((N + 127) / 128)), dim3(128), 0, s, out, nx, ny, nz, k,
                     alpha, L, q);
  return hipGetLastError();
}

hipError_t launch_embed(const double* goct, double* E, int comp, int nx, int ny, int nz, hipStream_t s) {
  const long long tot = 8LL * nx * ny * nz;
  hipLaunchKernelGGL(motgreen::k_embed, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, goct, E, comp, nx,
                     ny, nz);
  return hipGetLastError();
}

int compress_blocks(int nx, int ny, int nz) {
  const long long cnt = (long long)(nx + 1) * (ny + 1) * (nz + 1);
  return (int)((cnt + 255) / 256);
}

hipError_t launch_compress(const void* spec, double* lam64, float* lam32, double* imax, int comp, int nx,
                           int ny, int nz, int kxs, double scale, int w64, int w32, hipStream_t s) {
  hipLaunchKernelGGL(motgreen::k_compress, dim3(compress_blocks(nx, ny, nz)), dim3(256), 0, s,
                     (const double2*)spec, lam64, lam32, imax, comp, nx, ny, nz, kxs, scale, w64, w32);
  return hipGetLastError();
}

}  // namespace motimpl
