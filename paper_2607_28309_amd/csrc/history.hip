// History right-hand side of the MOT recursion (Eq. 3, Eq. 6):
//   S_{n+1}(k) = sum_{j=1..ell} Lambda_j(k) J^_{n+1-j}(k),
// accumulated pointwise over the spectra of past currents kept in a ring
// (slot t mod ell holds J^_t).  Each thread owns one octant frequency
// (kx, kyc, kzc); its up to four mirror points ky in {kyc, Py-kyc},
// kz in {kzc, Pz-kzc} share the six Lambda_j values (reflection signs: xy odd
// in ky, xz odd in kz, yz odd in both).
//
// Temporal blocking: at the start of a block of B steps (after J^_{n0} is
// pushed; B = 8, halved while B exceeds ell) one pass over the ring computes
// the contributions of all slots t <= n0 to the next B right-hand sides,
//   P_b = sum_{m>=0} Lambda_{m+b} J^_{n0-m},   b = 1..B,
// reading every slot and every Lambda_j once (a sliding window of B Lambda
// values is kept in registers).  Step n0+b-1 then adds only its b-1 newest
// lags, S_{n0+b} = P_b + sum_{j=1..b-1} Lambda_j J^_{n0+b-j}.  With B = 8 the
// block has a second level: at step n0+4 one pass of the same kind over the
// four slots n0+1..n0+4 adds their contributions to P_5..P_8 (the new P_5 is
// S_{n0+5}), so steps n0+5..n0+7 add at most their three newest lags.  The
// sums are the same as the plain per-step one, in another order.
#include <hip/hip_runtime.h>

#include "fft_core.h"
#include "mot_internal.h"

using motfft::cpx;

namespace motimpl {

struct Geo {
  int nx, ny, nz, kxs, nl;
};

// The mirror points of one octant frequency that a thread takes: NM = 4
// (both kz sides), NM = 2 (the kz side `side`, both ky sides) or NM = 1 (kz
// side side >> 1, ky side side & 1); mirror i is kz side a(i), ky side b(i).
template <int NM>
struct Point {
  size_t off[NM];
  bool keep[NM];
  int a[NM], b[NM];
};

//
// Frequencies are numbered along the padded rows (kx < kxs, the storage
// layout of the spectra and of Lambda), so that every wave reads whole
// 128-byte lines: a wave's frequencies start at a multiple of its width in
// that numbering.  Numbered along the used kx < nx + 1 instead, waves start
// anywhere in a row and the lines they share with the neighbouring
// workgroup, read at another time, are fetched from HBM twice.  The threads
// of the padding columns kx > nx return at once.
template <int NM>
__device__ __forceinline__ bool octant_point(const Geo& g, long long id, int side, size_t& lo, Point<NM>& pt) {
  const long long cnt = (long long)g.kxs * (g.ny + 1) * (g.nz + 1);
  if (id >= cnt) return false;
  const int kx = (int)(id % g.kxs), kyc = (int)((id / g.kxs) % (g.ny + 1)),
            kzc = (int)(id / ((long long)g.kxs * (g.ny + 1)));
  if (kx > g.nx) return false;
  const int py = 2 * g.ny, pz = 2 * g.nz;
  const size_t plane = (size_t)py * g.kxs;
  lo = ((size_t)kzc * (g.ny + 1) + kyc) * g.kxs + kx;
  const bool dupy = (kyc == 0 || kyc == g.ny), dupz = (kzc == 0 || kzc == g.nz);
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    const int a = NM == 4 ? i >> 1 : NM == 2 ? side : side >> 1, b = NM == 1 ? side & 1 : i & 1;
    const int kz = a ? pz - kzc : kzc, ky = b ? py - kyc : kyc;
    pt.off[i] = (size_t)(kz % pz) * plane + (size_t)(ky % py) * g.kxs + kx;
    pt.keep[i] = !((a && dupz) || (b && dupy));
    pt.a[i] = a;
    pt.b[i] = b;
  }
  return true;
}

// acc += Lambda J for one mirror point (signs sy, sz), one multiply-add per
// term into the accumulator.
template <typename T>
__device__ __forceinline__ void mac3(cpx<T> (&acc)[3], const T* l, T sy, T sz, cpx<T> jx, cpx<T> jy, cpx<T> jz) {
  const T xy = sy * l[3], xz = sz * l[4], yz = sy * sz * l[5];
  acc[0].x += l[0] * jx.x;
  acc[0].x += xy * jy.x;
  acc[0].x += xz * jz.x;
  acc[0].y += l[0] * jx.y;
  acc[0].y += xy * jy.y;
  acc[0].y += xz * jz.y;
  acc[1].x += xy * jx.x;
  acc[1].x += l[1] * jy.x;
  acc[1].x += yz * jz.x;
  acc[1].y += xy * jx.y;
  acc[1].y += l[1] * jy.y;
  acc[1].y += yz * jz.y;
  acc[2].x += xz * jx.x;
  acc[2].x += yz * jy.x;
  acc[2].x += l[2] * jz.x;
  acc[2].y += xz * jx.y;
  acc[2].y += yz * jy.y;
  acc[2].y += l[2] * jz.y;
}

// S = init + sum_{j=1..nrec} Lambda_j J^_{n+1-j}  (init may be null)
template <typename T>
__global__ __launch_bounds__(256) void k_mac_recent(const cpx<T>* __restrict__ ring, const T* __restrict__ lamh,
                                                    const cpx<T>* __restrict__ init, cpx<T>* __restrict__ out,
                                                    Geo g, long long n, int nrec) {
  size_t lo;
  Point<4> pt;
  if (!octant_point<4>(g, (long long)blockIdx.x * blockDim.x + threadIdx.x, 0, lo, pt)) return;
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

// P_b = init_b + sum_{m=0..nold-1} Lambda_{m+b} J^_{n0-m} for b = 1..B
// (Lambda_{>ell} = 0; init_b = iblk + (b-1) * slot, or 0 without iblk);
// P_1 -> out0, P_b -> pblk + (b-2) * slot for b >= 2.  NM = 4: a thread takes
// all four mirror points of its octant frequency; NM = 2 (for long blocks,
// whose B accumulators per point would not fit the registers): the two
// threads of a frequency take one kz side each and read the same Lambda
// words; NM = 1 (long blocks in FP64): four threads per frequency, one
// mirror point each.  Two waves per SIMD at least (a register budget of 256).
template <typename T, int B, int NM>
__global__ __launch_bounds__(256, 2) void k_mac_block(const cpx<T>* __restrict__ ring, const T* __restrict__ lamh,
                                                   cpx<T>* out0, cpx<T>* pblk, const cpx<T>* iblk, Geo g,
                                                   long long n0, int nold) {
  // octant frequencies per workgroup; with NM = 2 the two kz sides of a
  // frequency are neighbouring lanes of one wave, which read its Lambda words
  // with the same instruction
  constexpr int PER = 256 / (4 / NM);
  size_t lo;
  Point<NM> pt;
  const int t = (int)threadIdx.x;
  const long long id = (long long)blockIdx.x * PER + (NM == 4 ? t : NM == 2 ? t >> 1 : t >> 2);
  if (!octant_point<NM>(g, id, NM == 4 ? 0 : NM == 2 ? (t & 1) : (t & 3), lo, pt)) return;
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
  // With NM = 2 the kz sign sz is known only at run time (with NM = 1 the ky
  // sign sy too): the z (y) component of each loaded current is multiplied
  // by sz (sy) and the z (y) accumulators carry sz (sy) times their value
  // (sz^2 = sy^2 = 1), so that the B multiply-adds per load see compile-time
  // signs only.
  const T sz2 = NM <= 2 && pt.a[0] ? (T)-1 : (T)1;
  const T sy2 = NM == 1 && pt.b[0] ? (T)-1 : (T)1;
  cpx<T> acc[B][NM][3];
#pragma unroll
  for (int b = 0; b < B; ++b)
#pragma unroll
    for (int i = 0; i < NM; ++i) {
      if (iblk) {
        const cpx<T>* I = iblk + (size_t)b * slot;
        acc[b][i][0] = I[pt.off[i]];
        const cpx<T> y = I[comp + pt.off[i]];
        acc[b][i][1] = cpx<T>{sy2 * y.x, sy2 * y.y};
        const cpx<T> z = I[2 * comp + pt.off[i]];
        acc[b][i][2] = cpx<T>{sz2 * z.x, sz2 * z.y};
      } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[b][i][q] = cpx<T>{(T)0, (T)0};
      }
    }
  auto load_slot = [&](int m, cpx<T> (&jv)[NM][3]) {
    const cpx<T>* R = ring + (size_t)((n0 - m) % g.nl) * slot;
#pragma unroll
    for (int i = 0; i < NM; ++i)
#pragma unroll
      for (int q = 0; q < 3; ++q) jv[i][q] = R[q * comp + pt.off[i]];
  };
  // FP32: the next slot's currents and the next window value are loaded
  // before this slot's multiply-adds, so that their latency overlaps them
  // (FP64 has no registers to spare for it)
  constexpr bool PREFETCH = sizeof(T) == 4;
  cpx<T> jv[NM][3];
  if (PREFETCH && nold > 0) load_slot(0, jv);
  // the loop starts with no load in flight (vmcnt 0): the wait counts inside
  // the loop then follow its own loads only
  if constexpr (PREFETCH) __builtin_amdgcn_s_waitcnt(0x0F70);
  for (int m = 0; m < nold; ++m) {
    cpx<T> jn[NM][3];
    T ln[6];
    if constexpr (PREFETCH) {
      load_slot(m + 1 < nold ? m + 1 : m, jn);
      lam_at(m + 1 + B, ln);
    } else {
      load_slot(m, jv);
    }
    if constexpr (NM <= 2)
#pragma unroll
      for (int i = 0; i < NM; ++i) jv[i][2] = cpx<T>{sz2 * jv[i][2].x, sz2 * jv[i][2].y};
    if constexpr (NM == 1) jv[0][1] = cpx<T>{sy2 * jv[0][1].x, sy2 * jv[0][1].y};
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int i = 0; i < NM; ++i)
        mac3<T>(acc[b][i], w[b], (NM != 1 && (i & 1)) ? (T)-1 : (T)1, (NM == 4 && (i >> 1)) ? (T)-1 : (T)1,
                jv[i][0], jv[i][1], jv[i][2]);
#pragma unroll
    for (int b = 0; b + 1 < B; ++b)
#pragma unroll
      for (int c = 0; c < 6; ++c) w[b][c] = w[b + 1][c];
    if constexpr (PREFETCH) {
#pragma unroll
      for (int c = 0; c < 6; ++c) w[B - 1][c] = ln[c];
#pragma unroll
      for (int i = 0; i < NM; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) jv[i][q] = jn[i][q];
    } else {
      lam_at(m + 1 + B, w[B - 1]);
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) {
    cpx<T>* dst = b == 0 ? out0 : pblk + (size_t)(b - 1) * slot;
#pragma unroll
    for (int i = 0; i < NM; ++i)
      if (pt.keep[i]) {
        dst[pt.off[i]] = acc[b][i][0];
        dst[comp + pt.off[i]] = cpx<T>{sy2 * acc[b][i][1].x, sy2 * acc[b][i][1].y};
        dst[2 * comp + pt.off[i]] = cpx<T>{sz2 * acc[b][i][2].x, sz2 * acc[b][i][2].y};
      }
  }
}

static inline long long mac_count(const Geo& g) { return (long long)g.kxs * (g.ny + 1) * (g.nz + 1); }

static inline dim3 mac_grid(const Geo& g) { return dim3((unsigned)((mac_count(g) + 255) / 256)); }

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

hipError_t launch_mac_block(const void* ring, const void* lamh, void* out0, void* pblk, const void* iblk, int f64,
                            int B, int nl, long long n0, int nold, int nx, int ny, int nz, int kxs, hipStream_t s) {
  const Geo g{nx, ny, nz, kxs, nl};
  const dim3 gr = mac_grid(g);
  const long long cnt = mac_count(g);
  const dim3 gr2((unsigned)((cnt + 127) / 128));  // two threads per octant frequency
  const dim3 gr4((unsigned)((cnt + 63) / 64));    // four
#define LB(T, BB, NM, GR)                                                                                 \
  hipLaunchKernelGGL((k_mac_block<T, BB, NM>), GR, dim3(256), 0, s, (const cpx<T>*)ring, (const T*)lamh,   \
                     (cpx<T>*)out0, (cpx<T>*)pblk, (const cpx<T>*)iblk, g, n0, nold)
  if (f64) {
    if (B == 1) LB(double, 1, 4, gr);
    else if (B == 2) LB(double, 2, 4, gr);
    else if (B == 4) LB(double, 4, 2, gr2);
    else if (B == 8) LB(double, 8, 1, gr4);
    else return hipErrorInvalidValue;
  } else {
    if (B == 1) LB(float, 1, 4, gr);
    else if (B == 2) LB(float, 2, 4, gr);
    else if (B == 4) LB(float, 4, 4, gr);
    else if (B == 8) LB(float, 8, 2, gr2);
    else return hipErrorInvalidValue;
  }
#undef LB
  return hipGetLastError();
}

}  // namespace motimpl
