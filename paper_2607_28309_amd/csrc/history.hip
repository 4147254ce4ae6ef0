// History right-hand side of the MOT recursion (Eq. 3, Eq. 6):
//   S_{n+1}(k) = sum_{j=1..ell} Lambda_j(k) J^_{n+1-j}(k),
// accumulated pointwise over the spectra of past currents kept in a ring
// (slot t mod ell holds J^_t).  Each thread owns one octant frequency
// (kx, kyc, kzc); its up to four mirror points ky in {kyc, Py-kyc},
// kz in {kzc, Pz-kzc} share the six Lambda_j values (reflection signs: xy odd
// in ky, xz odd in kz, yz odd in both).
//
// Temporal blocking: at the start of a block of B steps (after J^_{n0} is
// pushed) one pass over the ring computes the contributions of all slots
// t <= n0 to the next B right-hand sides,
//   P_b = sum_{m>=0} Lambda_{m+b} J^_{n0-m},   b = 1..B,
// reading every slot and every Lambda_j once (a sliding window of B Lambda
// values is kept in registers).  Step n0+b-1 then adds only its b-1 newest
// lags, S_{n0+b} = P_b + sum_{j=1..b-1} Lambda_j J^_{n0+b-j}.  The sums are
// the same as the plain per-step one, in another order.
#include <hip/hip_runtime.h>

#include "fft_core.h"
#include "mot_internal.h"

using motfft::cpx;

namespace motimpl {

struct Geo {
  int nx, ny, nz, kxs, nl;
};

template <typename T>
struct Point {
  size_t off[4];
  bool keep[4];
};

template <typename T>
__device__ __forceinline__ bool octant_point(const Geo& g, size_t& lo, Point<T>& pt) {
  const long long cnt = (long long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= cnt) return false;
  const int kx = (int)(id % (g.nx + 1)), kyc = (int)((id / (g.nx + 1)) % (g.ny + 1)),
            kzc = (int)(id / ((long long)(g.nx + 1) * (g.ny + 1)));
  const int py = 2 * g.ny, pz = 2 * g.nz;
  const size_t plane = (size_t)py * g.kxs;
  lo = ((size_t)kzc * (g.ny + 1) + kyc) * g.kxs + kx;
  const bool dupy = (kyc == 0 || kyc == g.ny), dupz = (kzc == 0 || kzc == g.nz);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int a = i >> 1, b = i & 1;
    const int kz = a ? pz - kzc : kzc, ky = b ? py - kyc : kyc;
    pt.off[i] = (size_t)(kz % pz) * plane + (size_t)(ky % py) * g.kxs + kx;
    pt.keep[i] = !((a && dupz) || (b && dupy));
  }
  return true;
}

template <typename T>
__device__ __forceinline__ void mac3(cpx<T> (&acc)[3], const T* l, T sy, T sz, cpx<T> jx, cpx<T> jy, cpx<T> jz) {
  const T xy = sy * l[3], xz = sz * l[4], yz = sy * sz * l[5];
  acc[0].x += l[0] * jx.x + xy * jy.x + xz * jz.x;
  acc[0].y += l[0] * jx.y + xy * jy.y + xz * jz.y;
  acc[1].x += xy * jx.x + l[1] * jy.x + yz * jz.x;
  acc[1].y += xy * jx.y + l[1] * jy.y + yz * jz.y;
  acc[2].x += xz * jx.x + yz * jy.x + l[2] * jz.x;
  acc[2].y += xz * jx.y + yz * jy.y + l[2] * jz.y;
}

// S = init + sum_{j=1..nrec} Lambda_j J^_{n+1-j}  (init may be null)
template <typename T>
__global__ __launch_bounds__(256) void k_mac_recent(const cpx<T>* __restrict__ ring, const T* __restrict__ lamh,
                                                    const cpx<T>* __restrict__ init, cpx<T>* __restrict__ out,
                                                    Geo g, long long n, int nrec) {
  size_t lo;
  Point<T> pt;
  if (!octant_point<T>(g, lo, pt)) return;
  const size_t comp = (size_t)(2 * g.nz) * (2 * g.ny) * g.kxs;
  const size_t slot = 3 * comp;
  const size_t lcomp = (size_t)(g.nz + 1) * (g.ny + 1) * g.kxs;
  cpx<T> acc[4][3];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[i][q] = init ? init[q * comp + pt.off[i]] : cpx<T>{(T)0, (T)0};
  for (int j = 1; j <= nrec; ++j) {
    const cpx<T>* R = ring + (size_t)((n + 1 - j) % g.nl) * slot;
    const T* L = lamh + (size_t)(j - 1) * 6 * lcomp + lo;
    const T l[6] = {L[0], L[lcomp], L[2 * lcomp], L[3 * lcomp], L[4 * lcomp], L[5 * lcomp]};
#pragma unroll
    for (int i = 0; i < 4; ++i)
      mac3<T>(acc[i], l, (i & 1) ? (T)-1 : (T)1, (i >> 1) ? (T)-1 : (T)1, R[pt.off[i]], R[comp + pt.off[i]],
              R[2 * comp + pt.off[i]]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (pt.keep[i])
#pragma unroll
      for (int q = 0; q < 3; ++q) out[q * comp + pt.off[i]] = acc[i][q];
}

// P_b = sum_{m=0..nold-1} Lambda_{m+b} J^_{n0-m} for b = 1..B (Lambda_{>ell} = 0);
// P_1 -> out0, P_b -> pblk + (b-2) * slot for b >= 2.
template <typename T, int B>
__global__ __launch_bounds__(256) void k_mac_block(const cpx<T>* __restrict__ ring, const T* __restrict__ lamh,
                                                   cpx<T>* __restrict__ out0, cpx<T>* __restrict__ pblk, Geo g,
                                                   long long n0, int nold) {
  size_t lo;
  Point<T> pt;
  if (!octant_point<T>(g, lo, pt)) return;
  const size_t comp = (size_t)(2 * g.nz) * (2 * g.ny) * g.kxs;
  const size_t slot = 3 * comp;
  const size_t lcomp = (size_t)(g.nz + 1) * (g.ny + 1) * g.kxs;
  auto lam_at = [&](int lag, T* l) {
    if (lag > g.nl) {
#pragma unroll
      for (int c = 0; c < 6; ++c) l[c] = (T)0;
      return;
    }
    const T* L = lamh + (size_t)(lag - 1) * 6 * lcomp + lo;
#pragma unroll
    for (int c = 0; c < 6; ++c) l[c] = L[c * lcomp];
  };
  T w[B][6];  // window: w[b] = Lambda_{m+1+b}
#pragma unroll
  for (int b = 0; b < B; ++b) lam_at(b + 1, w[b]);
  cpx<T> acc[B][4][3];
#pragma unroll
  for (int b = 0; b < B; ++b)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[b][i][q] = cpx<T>{(T)0, (T)0};
  for (int m = 0; m < nold; ++m) {
    const cpx<T>* R = ring + (size_t)((n0 - m) % g.nl) * slot;
    cpx<T> jv[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 3; ++q) jv[i][q] = R[q * comp + pt.off[i]];
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        mac3<T>(acc[b][i], w[b], (i & 1) ? (T)-1 : (T)1, (i >> 1) ? (T)-1 : (T)1, jv[i][0], jv[i][1], jv[i][2]);
#pragma unroll
    for (int b = 0; b + 1 < B; ++b)
#pragma unroll
      for (int c = 0; c < 6; ++c) w[b][c] = w[b + 1][c];
    lam_at(m + 1 + B, w[B - 1]);
  }
#pragma unroll
  for (int b = 0; b < B; ++b) {
    cpx<T>* dst = b == 0 ? out0 : pblk + (size_t)(b - 1) * slot;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (pt.keep[i])
#pragma unroll
        for (int q = 0; q < 3; ++q) dst[q * comp + pt.off[i]] = acc[b][i][q];
  }
}

static inline dim3 mac_grid(const Geo& g) {
  const long long cnt = (long long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
  return dim3((unsigned)((cnt + 255) / 256));
}

hipError_t launch_mac_recent(const void* ring, const void* lamh, const void* init, void* out, int f64, int nl,
                             long long n, int nrec, int nx, int ny, int nz, int kxs, hipStream_t s) {
  const Geo g{nx, ny, nz, kxs, nl};
  if (f64)
    hipLaunchKernelGGL(k_mac_recent<double>, mac_grid(g), dim3(256), 0, s, (const cpx<double>*)ring,
                       (const double*)lamh, (const cpx<double>*)init, (cpx<double>*)out, g, n, nrec);
  else
    hipLaunchKernelGGL(k_mac_recent<float>, mac_grid(g), dim3(256), 0, s, (const cpx<float>*)ring,
                       (const float*)lamh, (const cpx<float>*)init, (cpx<float>*)out, g, n, nrec);
  return hipGetLastError();
}

hipError_t launch_mac_block(const void* ring, const void* lamh, void* out0, void* pblk, int f64, int B, int nl,
                            long long n0, int nold, int nx, int ny, int nz, int kxs, hipStream_t s) {
  const Geo g{nx, ny, nz, kxs, nl};
  const dim3 gr = mac_grid(g);
#define LB(T, BB)                                                                                       \
  hipLaunchKernelGGL((k_mac_block<T, BB>), gr, dim3(256), 0, s, (const cpx<T>*)ring, (const T*)lamh,     \
                     (cpx<T>*)out0, (cpx<T>*)pblk, g, n0, nold)
  if (f64) {
    if (B == 1) LB(double, 1);
    else if (B == 2) LB(double, 2);
    else return hipErrorInvalidValue;
  } else {
    if (B == 1) LB(float, 1);
    else if (B == 2) LB(float, 2);
    else if (B == 4) LB(float, 4);
    else return hipErrorInvalidValue;
  }
#undef LB
  return hipGetLastError();
}

}  // namespace motimpl
