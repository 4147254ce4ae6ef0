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

// Word 3 of a raw (untyped, stride 0) buffer resource on gfx9-family parts:
// 32-bit data format, no swizzle; loads past num_records return zero.
constexpr int BUF_WORD3 = 0x00020000;

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
template <typename T, int B, int NM, bool O32 = false>
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
  // With NM = 2 the kz sign sz of a thread's points is known only at run time
  // (with NM = 1 the ky sign sy too).  It goes into the window's copies of the
  // off-diagonal Lambda components that it multiplies (xy by sy, xz by sz, yz
  // by sy sz), so that the multiply-adds see compile-time signs only.  A
  // product of two values one of which changed sign is exactly the negated
  // product: the sums are those of the plain formula.
  const T sz2 = NM <= 2 && pt.a[0] ? (T)-1 : (T)1;
  const T sy2 = NM == 1 && pt.b[0] ? (T)-1 : (T)1;
  auto fold_signs = [&](T* l) {
    if constexpr (NM == 1) {
      l[3] *= sy2;
      l[5] *= sy2 * sz2;
    }
    if constexpr (NM <= 2) {
      l[4] *= sz2;
      if constexpr (NM == 2) l[5] *= sz2;
    }
  };
  auto lam_at = [&](int lag, T* l) {
    if (lag > g.nl) {
#pragma unroll
      for (int c = 0; c < 6; ++c) l[c] = (T)0;
      return;
    }
    const T* L = lamh + (size_t)(lag - 1) * 6 * lcomp + lo;
#pragma unroll
    for (int c = 0; c < 6; ++c) l[c] = L[c * lcomp];
    fold_signs(l);
  };
  T w[B][6];  // window: w[b] = Lambda_{m+1+b}
#pragma unroll
  for (int b = 0; b < B; ++b) lam_at(b + 1, w[b]);
  cpx<T> acc[B][NM][3];
#pragma unroll
  for (int b = 0; b < B; ++b)
#pragma unroll
    for (int i = 0; i < NM; ++i) {
      if (iblk) {
        const cpx<T>* I = iblk + (size_t)b * slot;
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[b][i][q] = I[q * comp + pt.off[i]];
      } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[b][i][q] = cpx<T>{(T)0, (T)0};
      }
    }
  // ring slot of J^_{n0-m} for 0 <= m < nl: one 64-bit remainder per thread,
  // then 32-bit steps
  const int s0 = (int)(n0 % g.nl);
  // One slot: its multiply-adds with the window, then the window moves on
  // (w[B - 1] = the next Lambda value, ln, or 0 past the last lag).
  auto mac_slot = [&](const cpx<T> (&jv)[NM][3], const T (&ln)[6], bool lzero) {
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
#pragma unroll
    for (int c = 0; c < 6; ++c) w[B - 1][c] = lzero ? (T)0 : ln[c];
  };
  if constexpr (sizeof(T) == 4) {
    // FP32: NS register sets of currents take the slots in turn (slot m in
    // set m mod NS).  The work on slot m first issues the loads of slot
    // m + NS - 1 (and of the Lambda value as many slots ahead) into the set
    // that slot m - 1 has just released, then does slot m's multiply-adds:
    // every load has NS - 1 slots of multiply-adds to arrive in (with two
    // waves per SIMD, one slot is about 1.2 k cycles of each wave's issue).
    // No load in the loop is conditional, so that no register with a load in
    // flight is merged or copied at a branch or at the loop's back edge.  A
    // loop trip takes U slots (all set indices compile-time); the last
    // nold mod U slots follow, each behind a wave-uniform test.
    //
    // With O32 (a slot and a lag's six Lambda components each within 4 GiB)
    // the loads are buffer loads: a wave-uniform resource per slot and lag
    // (scalar registers) and per-thread 32-bit byte offsets that stay fixed
    // over the slots, so that no address arithmetic is redone per slot.  A
    // slot m >= nold and a lag past the last get an empty range, whose loads
    // return zero without touching memory: no select zeroes the lags past
    // the last, and the loads ahead of the last slots need no clamp.  Without
    // O32 the indices are clamped to valid slots and lags and the window
    // zeroes the lags past the last.
    //
    // Four sets with two mirror points per thread and 32-bit offsets, else
    // three (the registers of a fourth set would spill).
    constexpr int NS = O32 && NM == 2 ? 4 : 3;
    const int last = nold > 0 ? nold - 1 : 0;
    unsigned jo[NM][3], lof[6];
    if constexpr (O32) {
#pragma unroll
      for (int i = 0; i < NM; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) jo[i][q] = (unsigned)((q * comp + pt.off[i]) * sizeof(cpx<T>));
#pragma unroll
      for (int c = 0; c < 6; ++c) lof[c] = (unsigned)((c * lcomp + lo) * sizeof(T));
    }
    auto ld_slot = [&](int m, cpx<T> (&jv)[NM][3]) {
      const int mc = m < last ? m : last;
      const int sl = s0 - mc < 0 ? s0 - mc + g.nl : s0 - mc;
      const cpx<T>* R = ring + (size_t)sl * slot;
      if constexpr (O32) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)R, (short)0, m < nold ? (int)(unsigned)(slot * sizeof(cpx<T>)) : 0, BUF_WORD3);
#pragma unroll
        for (int i = 0; i < NM; ++i)
#pragma unroll
          for (int q = 0; q < 3; ++q)
            jv[i][q] = __builtin_bit_cast(cpx<T>, __builtin_amdgcn_raw_buffer_load_b64(rs, jo[i][q], 0, 0));
      } else {
#pragma unroll
        for (int i = 0; i < NM; ++i)
#pragma unroll
          for (int q = 0; q < 3; ++q) jv[i][q] = R[q * comp + pt.off[i]];
      }
    };
    auto ld_lam = [&](int lag, T (&l)[6]) {
      const T* L = lamh + (size_t)((lag < g.nl ? lag : g.nl) - 1) * 6 * lcomp;
      if constexpr (O32) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)L, (short)0, lag <= g.nl ? (int)(unsigned)(6 * lcomp * sizeof(T)) : 0, BUF_WORD3);
#pragma unroll
        for (int c = 0; c < 6; ++c) l[c] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, lof[c], 0, 0));
      } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) l[c] = L[c * lcomp + lo];
      }
    };
    cpx<T> js[NS][NM][3];
#pragma unroll
    for (int k = 0; k + 1 < NS; ++k) ld_slot(k, js[k]);
    if constexpr (O32 && NM == 2) {
      // Lambda in place: the window rotates through NL >= B + NS register
      // sets (NL a multiple of NS, U = NL): lag m + j (m a multiple of NL)
      // sits in set j mod NL, so that every window access has a compile-time
      // set and no value is copied.  Step k overwrites the set of lag
      // m + k + NS + B - NL <= m + k, whose last use was step k - 1 at the
      // latest, with lag m + k + NS + B.  The kz sign goes into the xz and yz
      // components of lag m + k + 1 + B after the multiply-adds of step k
      // (the lags of the first window come folded), NS - 1 slots after its
      // load was issued and before its first use.
      constexpr int NL = (B + NS + NS - 1) / NS * NS;
      constexpr int U = NL;
      T lp[NL][6];
#pragma unroll
      for (int j = 1; j <= B; ++j)
#pragma unroll
        for (int c = 0; c < 6; ++c) lp[j % NL][c] = w[j - 1][c];
#pragma unroll
      for (int k = 0; k + 1 < NS; ++k) ld_lam(k + 1 + B, lp[(k + 1 + B) % NL]);
      auto step = [&](int m, int k) {
        ld_slot(m + NS - 1, js[(k + NS - 1) % NS]);
        ld_lam(m + NS + B, lp[(k + NS + B) % NL]);
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
          for (int i = 0; i < NM; ++i)
            mac3<T>(acc[b][i], lp[(k + 1 + b) % NL], (i & 1) ? (T)-1 : (T)1, (T)1, js[k % NS][i][0],
                    js[k % NS][i][1], js[k % NS][i][2]);
        fold_signs(lp[(k + 1 + B) % NL]);
      };
      const int nfull = nold / U * U;
      for (int m = 0; m < nfull; m += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) step(m + k, k);
      }
#pragma unroll
      for (int k = 0; k + 1 < U; ++k) {
        if (nfull + k >= nold) break;
        step(nfull + k, k);
      }
    } else {
      // Lambda through the shifting window: NS sets receive the loads
      // ahead, and each step moves one into w[B - 1].  A loop trip takes
      // U = B slots when B is a multiple of NS (the window is then back in
      // the registers it started in: no moves for its shifts), else NS.
      constexpr int U = B % NS == 0 ? B : NS;
      T ls[NS][6];
#pragma unroll
      for (int k = 0; k + 1 < NS; ++k) ld_lam(k + 1 + B, ls[k]);
      auto step = [&](int m, int k) {
        ld_slot(m + NS - 1, js[(k + NS - 1) % NS]);
        ld_lam(m + NS + B, ls[(k + NS - 1) % NS]);
        T l[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) l[c] = ls[k % NS][c];
        fold_signs(l);
        mac_slot(js[k % NS], l, !O32 && m + 1 + B > g.nl);
      };
      const int nfull = nold / U * U;
      for (int m = 0; m < nfull; m += U) {
#pragma unroll
        for (int k = 0; k < U; ++k) step(m + k, k);
      }
#pragma unroll
      for (int k = 0; k + 1 < U; ++k) {
        if (nfull + k >= nold) break;
        step(nfull + k, k);
      }
    }
  } else {
    // FP64 has no registers to spare for loads ahead
    for (int m = 0; m < nold; ++m) {
      cpx<T> jv[NM][3];
      T ln[6];
      const int sl = s0 - m < 0 ? s0 - m + g.nl : s0 - m;
      const cpx<T>* R = ring + (size_t)sl * slot;
#pragma unroll
      for (int i = 0; i < NM; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) jv[i][q] = R[q * comp + pt.off[i]];
      lam_at(m + 1 + B, ln);
      mac_slot(jv, ln, false);
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) {
    cpx<T>* dst = b == 0 ? out0 : pblk + (size_t)(b - 1) * slot;
#pragma unroll
    for (int i = 0; i < NM; ++i)
      if (pt.keep[i]) {
#pragma unroll
        for (int q = 0; q < 3; ++q) dst[q * comp + pt.off[i]] = acc[b][i][q];
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
                            int B, int nl, long long n0, int nold, int nx, int ny, int nz, int kxs, hipStream_t s,
                            int wide) {
  const Geo g{nx, ny, nz, kxs, nl};
  const dim3 gr = mac_grid(g);
  const long long cnt = mac_count(g);
  const dim3 gr2((unsigned)((cnt + 127) / 128));  // two threads per octant frequency
  const dim3 gr4((unsigned)((cnt + 63) / 64));    // four
  // 32-bit per-thread offsets when a slot of the ring and a lag of Lambda
  // each fit in 4 GiB (FP32 only)
  const size_t comp = (size_t)(2 * nz) * (2 * ny) * kxs, lcomp = (size_t)(nz + 1) * (ny + 1) * kxs;
  const bool o32 =
      !wide && 3 * comp * sizeof(cpx<float>) <= 0xFFFFFFFFull && 6 * lcomp * sizeof(float) <= 0xFFFFFFFFull;
#define LB(T, BB, NM, GR, O)                                                                              \
  hipLaunchKernelGGL((k_mac_block<T, BB, NM, O>), GR, dim3(256), 0, s, (const cpx<T>*)ring, (const T*)lamh, \
                     (cpx<T>*)out0, (cpx<T>*)pblk, (const cpx<T>*)iblk, g, n0, nold)
#define LBF(BB, NM, GR)              \
  if (o32) LB(float, BB, NM, GR, true); \
  else LB(float, BB, NM, GR, false)
  if (f64) {
    if (B == 1) LB(double, 1, 4, gr, false);
    else if (B == 2) LB(double, 2, 4, gr, false);
    else if (B == 4) LB(double, 4, 2, gr2, false);
    else if (B == 8) LB(double, 8, 1, gr4, false);
    else return hipErrorInvalidValue;
  } else {
    if (B == 1) { LBF(1, 4, gr); }
    else if (B == 2) { LBF(2, 4, gr); }
    else if (B == 4) { LBF(4, 4, gr); }
    else if (B == 8) { LBF(8, 2, gr2); }
    else return hipErrorInvalidValue;
  }
#undef LBF
#undef LB
  return hipGetLastError();
}

// ---- History by FFTs in time (FP32 ring) ----------------------------------
//
// The lags beyond the current time block are applied block by block in the
// frequency domain of time.  Steps are grouped in blocks of S = TF_S; at the
// push of J^_n with n = beta S, the right-hand sides of steps n + 1 + i,
// i = 0..S-1, receive from the currents of block m (times
// t = (beta - m) S + 1 + q, q = 0..S-1) the lags L = m S + i - q, which lie
// in (m-1) S + 1 .. (m+1) S - 1.  With x_m[q] = J^_t zero-padded to 2S and
// k_m[d] = Lambda_{(m-1) S + d} (d = 1..2S-1, k_m[0] = 0), that sum is the
// entry S + i of the cyclic convolution of length 2S (no index wraps), so
//   far_i = IDFT_2S( sum_m K_m . X_m )[S + i],  K_m = DFT_2S(k_m), X_m = DFT_2S(x_m).
// Block m = 1 ends at n itself.  The lags inside the current block (the
// currents of steps beta S + 1 .. n' - 1 for step n') are left to the blocked
// multiply-accumulate above, which takes far as its initial value.
//
// Each workgroup takes 32 consecutive octant frequencies (numbered over the
// used kx of the octant rows, so that no lane idles on padding columns) at
// one mirror side, and all three components.  Per earlier block m, thread
// (component j, point p, parity h) transforms its current at the
// frequencies w = 2u + h, u = 0..31, as a 32-point DFT of x[q] W_64^{hq}
// (the two parities split the 64-point transform, whose upper inputs are
// zero), and the spectra go through LDS to thread (point p, group
// fg = 2j + h), which owns the frequencies w' = fg + 6r <= S and their
// partners 2S - w': it loads the six components of K_m(w') once for both
// (K_m is real in time, so K_m(2S - w) = conj K_m(w) and only w = 0..S are
// stored) and accumulates Y_i = sum_j K_m,ij X_m,j.  After the last block Y
// goes back through LDS, each parity is inverted (a 32-point inverse DFT),
// and the two parities of a point combine through a lane exchange:
//   y[S + i] = (E(i) - W_64^{-i} O(i)) / 2S.
// K is shared by the four mirror points of an octant frequency (reflection
// signs as in mac3); the four workgroups of one tile are neighbours in the
// XCD-aware order, so they read K through one L2.

struct Tw64 {
  // cos(2 pi j / 64); sin(2 pi j / 64) = cos(2 pi (j - 16) / 64)
  static constexpr double c[64] = {1, 0.99518472667219693, 0.98078528040323043, 0.95694033573220882, 0.92387953251128674, 0.88192126434835505, 0.83146961230254524, 0.77301045336273699, 0.70710678118654757, 0.63439328416364549, 0.55557023301960229, 0.47139673682599781, 0.38268343236508984, 0.29028467725446233, 0.19509032201612833, 0.09801714032956077, 6.123233995736766e-17, -0.098017140329560645, -0.19509032201612819, -0.29028467725446216, -0.38268343236508973, -0.4713967368259977, -0.55557023301960196, -0.63439328416364538, -0.70710678118654746, -0.77301045336273699, -0.83146961230254535, -0.88192126434835494, -0.92387953251128674, -0.95694033573220882, -0.98078528040323043, -0.99518472667219682, -1, -0.99518472667219693, -0.98078528040323043, -0.95694033573220894, -0.92387953251128685, -0.88192126434835505, -0.83146961230254546, -0.7730104533627371, -0.70710678118654768, -0.63439328416364593, -0.55557023301960218, -0.47139673682599786, -0.38268343236509034, -0.29028467725446244, -0.19509032201612866, -0.098017140329560451, -1.8369701987210297e-16, 0.09801714032956009, 0.1950903220161283, 0.29028467725446205, 0.38268343236509, 0.47139673682599759, 0.55557023301960184, 0.6343932841636456, 0.70710678118654735, 0.77301045336273666, 0.83146961230254524, 0.88192126434835483, 0.92387953251128652, 0.95694033573220882, 0.98078528040323032, 0.99518472667219693};
  static constexpr double cs(int j) { return c[j & 63]; }
  static constexpr double sn(int j) { return c[(j + 48) & 63]; }
};

__constant__ double tf_cos64[64] = {1, 0.99518472667219693, 0.98078528040323043, 0.95694033573220882, 0.92387953251128674, 0.88192126434835505, 0.83146961230254524, 0.77301045336273699, 0.70710678118654757, 0.63439328416364549, 0.55557023301960229, 0.47139673682599781, 0.38268343236508984, 0.29028467725446233, 0.19509032201612833, 0.09801714032956077, 6.123233995736766e-17, -0.098017140329560645, -0.19509032201612819, -0.29028467725446216, -0.38268343236508973, -0.4713967368259977, -0.55557023301960196, -0.63439328416364538, -0.70710678118654746, -0.77301045336273699, -0.83146961230254535, -0.88192126434835494, -0.92387953251128674, -0.95694033573220882, -0.98078528040323043, -0.99518472667219682, -1, -0.99518472667219693, -0.98078528040323043, -0.95694033573220894, -0.92387953251128685, -0.88192126434835505, -0.83146961230254546, -0.7730104533627371, -0.70710678118654768, -0.63439328416364593, -0.55557023301960218, -0.47139673682599786, -0.38268343236509034, -0.29028467725446244, -0.19509032201612866, -0.098017140329560451, -1.8369701987210297e-16, 0.09801714032956009, 0.1950903220161283, 0.29028467725446205, 0.38268343236509, 0.47139673682599759, 0.55557023301960184, 0.6343932841636456, 0.70710678118654735, 0.77301045336273666, 0.83146961230254524, 0.88192126434835483, 0.92387953251128652, 0.95694033573220882, 0.98078528040323032, 0.99518472667219693};

// In-register DFT of length 32, in place: for inputs v[j] in natural order,
// X[k] = sum_j v[j] exp(-+2 pi i jk/32) ends up in v[tf_pos(k)].  32 = 8 x 4:
// inputs j = 4 j1 + j2, outputs k = k1 + 8 k2; length-8 transforms over j1,
// rotations W_32^{j2 k1}, length-4 transforms over j2 (no temporary copy of
// the 32 values, so that two such arrays and the loads fit the registers).
__device__ __forceinline__ constexpr int tf_pos(int k) { return 4 * (k & 7) + (k >> 3); }

template <bool INV>
__device__ __forceinline__ void dft32(cpx<float> (&v)[32]) {
#pragma unroll
  for (int j2 = 0; j2 < 4; ++j2) {
    cpx<float> a[8];
#pragma unroll
    for (int j1 = 0; j1 < 8; ++j1) a[j1] = v[4 * j1 + j2];
    motfft::Dft<8, INV, float>::run(a);
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
      const int e = 2 * j2 * k1;  // W_32^{j2 k1} = W_64^{2 j2 k1}
      if (e == 0) {
        v[4 * k1 + j2] = a[k1];
      } else {
        const float cr = (float)Tw64::cs(e), si = INV ? (float)Tw64::sn(e) : -(float)Tw64::sn(e);
        v[4 * k1 + j2] = motfft::cmul(a[k1], cpx<float>{cr, si});
      }
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 8; ++k1) motfft::Dft<4, INV, float>::run(&v[4 * k1]);
}

// K_m(w) = sum_{d=1..2S-1} Lambda_{(m-1)S+d} exp(-2 pi i w d / 2S) in FP64 from
// the stored Lambda (Lambda_L = 0 for L > nl); one thread per (octant point,
// component, m), all S + 1 frequencies.
__global__ __launch_bounds__(256) void k_tfft_prep(const float* __restrict__ lamh, cpx<float>* __restrict__ K,
                                                   long long lcomp, int nl, int M) {
  constexpr int S = TF_S;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= lcomp * 6 * M) return;
  const long long lo = id % lcomp;
  const int c = (int)((id / lcomp) % 6), m = (int)(id / (lcomp * 6)) + 1;
  double re[S + 1], im[S + 1];
#pragma unroll
  for (int w = 0; w <= S; ++w) re[w] = im[w] = 0.0;
  for (int d = 1; d < 2 * S; ++d) {
    const int L = (m - 1) * S + d;
    if (L > nl) break;
    const double v = (double)lamh[((size_t)(L - 1) * 6 + c) * lcomp + lo];
#pragma unroll
    for (int w = 0; w <= S; ++w) {
      const int e = (w * d) & 63;
      re[w] += v * tf_cos64[e];
      im[w] -= v * tf_cos64[(e + 48) & 63];
    }
  }
#pragma unroll
  for (int w = 0; w <= S; ++w)
    K[((size_t)((m - 1) * 6 + c) * (S + 1) + w) * lcomp + lo] = cpx<float>{(float)re[w], (float)im[w]};
}

// LDS index of X_j(2u + h) of point p: the two parities of a half-wave land
// on different banks
__device__ __forceinline__ int tf_lds(int j, int h, int u, int p) { return (j * 32 + u) * 64 + h * 32 + (p ^ (h << 4)); }

__global__ __launch_bounds__(192, 3) void k_tfft_far(const cpx<float>* __restrict__ ring, const cpx<float>* __restrict__ K,
                                                     cpx<float>* __restrict__ far, Geo g, long long n, int M, int nlog) {
  constexpr int S = TF_S;
  __shared__ cpx<float> xs[3 * 32 * 64];
  // logical tile: (32 consecutive octant frequencies in the numbering
  // f = (kzc (ny+1) + kyc)(nx+1) + kx over the used kx, mirror), mirror
  // fastest; tiles go to the XCDs in contiguous ranges (ids are dealt to
  // the 8 XCDs in turn)
  const int q8 = (nlog + 7) / 8;
  const int t = (int)(blockIdx.x % 8) * q8 + (int)(blockIdx.x / 8);
  if (t >= nlog) return;
  const int mu = t & 3, a = mu >> 1, b = mu & 1;
  const int kxu = g.nx + 1;
  const long long ftot = (long long)(g.nz + 1) * (g.ny + 1) * kxu;
  const long long f0 = (long long)(t >> 2) * 32;
  {
    // a tile whose rows are all duplicate mirrors (kz or ky on its own
    // mirror plane) has nothing to do
    const long long f1 = f0 + 31 < ftot ? f0 + 31 : ftot - 1;
    bool any = false;
    for (long long r = f0 / kxu; r <= f1 / kxu; ++r) {
      const int yc = (int)(r % (g.ny + 1)), zc = (int)(r / (g.ny + 1));
      any = any || !((a && (zc == 0 || zc == g.nz)) || (b && (yc == 0 || yc == g.ny)));
    }
    if (!any) return;
  }
  const int py = 2 * g.ny, pz = 2 * g.nz;
  // transforms: thread (component j, point p, parity h); products: thread
  // (point p, frequency group fg = 2 j + h), which owns the frequencies
  // w' = fg + 6 r <= S and their partners 2S - w'
  const int j = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63, p = lane >> 1, h = lane & 1;
  const int fg = 2 * j + h;
  const long long f = f0 + p;
  const long long orow = f / kxu;
  const int kx = (int)(f - orow * kxu);
  const int kyc = (int)(orow % (g.ny + 1)), kzc = (int)(orow / (g.ny + 1));
  const bool act = f < ftot && !((a && (kzc == 0 || kzc == g.nz)) || (b && (kyc == 0 || kyc == g.ny)));
  const int kz = a ? pz - kzc : kzc, ky = b ? py - kyc : kyc;
  const size_t comp = (size_t)pz * py * g.kxs;
  const size_t slot_bytes = 3 * comp * sizeof(cpx<float>);
  const size_t lcomp = (size_t)(g.nz + 1) * (g.ny + 1) * g.kxs;
  // byte offsets below 4 GiB from a wave-uniform base: one ring slot (3
  // components) and one (m, component) plane of K (S + 1 frequencies; the
  // plane's base is added in 64 bits)
  const unsigned roff = act ? (unsigned)(((size_t)j * comp + ((size_t)kz * py + ky) * g.kxs + kx) * sizeof(cpx<float>)) : 0u;
  const unsigned loff = act ? (unsigned)((((size_t)kzc * (g.ny + 1) + kyc) * g.kxs + kx) * sizeof(cpx<float>)) : 0u;
  const unsigned lstride = (unsigned)(lcomp * sizeof(cpx<float>));
  // reflection signs of the xy, xz, yz components at this mirror point
  const float sxy = b ? -1.f : 1.f, sxz = a ? -1.f : 1.f, syz = sxy * sxz;
  const long long beta = n / S;
  const int mmax = (int)(beta + 1 < M ? beta + 1 : M);
  cpx<float> acc[6][2][3];  // Y_i at w' = fg + 6 r (e = 0) and 2S - w' (e = 1)
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[r][e][i] = cpx<float>{0.f, 0.f};
  for (int m = 1; m <= mmax; ++m) {
    // currents of times t0 .. t0 + S - 1 (uniform across the workgroup)
    const long long t0 = (beta - m) * S + 1;
    const long long tlo = t0 > n - g.nl + 1 ? t0 : n - g.nl + 1;  // oldest time the ring still holds
    const long long tfirst = tlo > 0 ? tlo : 0;
    const int q0 = (int)(tfirst - t0);  // first q the ring holds (0..S)
    // slot of time t0 + q: sl0 + q, wrapped once at q = qw
    const int sl0 = (int)(((t0 % g.nl) + g.nl) % g.nl), qw = g.nl - sl0;
    const char* rb = (const char*)ring;
    // wave-uniform slot address plus the lane's 32-bit offset; idle lanes
    // (past the last frequency, or on a duplicate mirror) read offset 0 and
    // store nothing
    // every slot read is a valid one; times the ring no longer holds (or
    // before step 0) are zeroed afterwards, on a branch taken only by the
    // first blocks of a march
    cpx<float> x[32];
    const char* pq = rb + (size_t)sl0 * slot_bytes;
#pragma unroll
    for (int q = 0; q < S; ++q) {
      x[q] = *(const cpx<float>*)(pq + roff);
      pq = q + 1 == qw ? rb : pq + slot_bytes;
    }
    if (q0 > 0) {
#pragma unroll
      for (int q = 0; q < S; ++q)
        if (q < q0) x[q] = cpx<float>{0.f, 0.f};
    }
    // odd frequencies: x[q] W_64^q, then a 32-point DFT
#pragma unroll
    for (int q = 1; q < S; ++q) {
      const cpx<float> rr = motfft::cmul(x[q], cpx<float>{(float)Tw64::cs(q), -(float)Tw64::sn(q)});
      x[q] = h ? rr : x[q];
    }
    dft32<false>(x);
    __syncthreads();  // the previous block's reads of xs are done
#pragma unroll
    for (int u = 0; u < 32; ++u) xs[tf_lds(j, h, u, p)] = x[tf_pos(u)];
    __syncthreads();
    // Y_i(w) += sum_j K_m,ij(w) X_m,j(w): the six components of K_m(w') are
    // loaded once for w' and its partner 2S - w' (conjugate)
    const char* Kb = (const char*)(K + (size_t)(m - 1) * 6 * (S + 1) * lcomp);
    // (opaque per block: the addresses are formed here rather than held in
    // registers across the loop)
    unsigned ls = lstride, lof = loff;
    int fgm = fg;
    asm volatile("" : "+s"(ls));
    asm volatile("" : "+v"(lof));
    asm volatile("" : "+v"(fgm));
    // two halves of three frequency pairs: the 18 loads of a half are issued
    // together (no branch between them; w' > S reads w' = S and is dropped)
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      // (idle lanes read offset 0)
      cpx<float> kk[3][6];
#pragma unroll
      for (int rr = 0; rr < 3; ++rr) {
        const int wp = fgm + 6 * (3 * hf + rr);
        const unsigned wl = (unsigned)(wp <= S ? wp : S);
#pragma unroll
        for (int c = 0; c < 6; ++c) kk[rr][c] = *(const cpx<float>*)(Kb + (size_t)c * (S + 1) * lstride + (wl * ls + lof));
      }
#pragma unroll
      for (int rr = 0; rr < 3; ++rr) {
        const int r = 3 * hf + rr;
        const int wp = fgm + 6 * r;
        if (wp > S) continue;
        cpx<float> k6[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) k6[c] = kk[rr][c];
        k6[3] = cpx<float>{k6[3].x * sxy, k6[3].y * sxy};
        k6[4] = cpx<float>{k6[4].x * sxz, k6[4].y * sxz};
        k6[5] = cpx<float>{k6[5].x * syz, k6[5].y * syz};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          if (e == 1 && (wp == 0 || wp == S)) continue;
          const int w = e ? 2 * S - wp : wp;
          const float cs = e ? -1.f : 1.f;  // K(2S - w') = conj K(w')
          cpx<float> xv[3];
#pragma unroll
          for (int jj = 0; jj < 3; ++jj) xv[jj] = xs[tf_lds(jj, w & 1, w >> 1, p)];
          // rows (xx xy xz), (xy yy yz), (xz yz zz)
          const int ci[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
              // four multiply-adds per complex product, accumulated in order
              const cpx<float> kv = k6[ci[i][jj]];
              const float ky_ = cs * kv.y;
              acc[r][e][i].x = fmaf(kv.x, xv[jj].x, acc[r][e][i].x);
              acc[r][e][i].x = fmaf(-ky_, xv[jj].y, acc[r][e][i].x);
              acc[r][e][i].y = fmaf(kv.x, xv[jj].y, acc[r][e][i].y);
              acc[r][e][i].y = fmaf(ky_, xv[jj].x, acc[r][e][i].y);
            }
        }
      }
    }
  }
  // Y back through LDS to the transform layout, one inverse per parity, then
  // y[S + i] = (E(i) - W_64^{-i} O(i)) / 2S: the even lane writes i < 16,
  // the odd lane i >= 16
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    const int wp = fg + 6 * r;
    if (wp > S) continue;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      if (e == 1 && (wp == 0 || wp == S)) continue;
      const int w = e ? 2 * S - wp : wp;
#pragma unroll
      for (int i = 0; i < 3; ++i) xs[tf_lds(i, w & 1, w >> 1, p)] = acc[r][e][i];
    }
  }
  __syncthreads();
  cpx<float> y[32];
#pragma unroll
  for (int u = 0; u < 32; ++u) y[u] = xs[tf_lds(j, h, u, p)];
  dft32<true>(y);
  const float inv = 1.f / (2 * S);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const cpx<float> lo_ = y[tf_pos(u)], hi_ = y[tf_pos(16 + u)];
    const cpx<float> send = h ? lo_ : hi_;
    const cpx<float> recv{__shfl_xor(send.x, 1), __shfl_xor(send.y, 1)};
    const cpx<float> e = h ? recv : lo_, o = h ? hi_ : recv;
    // both rotations with literal constants, then the lane's one (a select
    // of the constants would become a table read)
    const cpx<float> wo0 = motfft::cmul(o, cpx<float>{(float)Tw64::cs(u), (float)Tw64::sn(u)});
    const cpx<float> wo1 = motfft::cmul(o, cpx<float>{(float)Tw64::cs(16 + u), (float)Tw64::sn(16 + u)});
    const cpx<float> wo = h ? wo1 : wo0;
    if (act)
      *(cpx<float>*)((char*)far + (size_t)(u + 16 * h) * slot_bytes + roff) =
          cpx<float>{(e.x - wo.x) * inv, (e.y - wo.y) * inv};
  }
}

hipError_t launch_tfft_prep(const float* lamh, void* K, int nl, int nx, int ny, int nz, int kxs, hipStream_t s) {
  const long long lcomp = (long long)(nz + 1) * (ny + 1) * kxs;
  const int M = tfft_blocks(nl);
  const long long cnt = lcomp * 6 * M;
  hipLaunchKernelGGL(k_tfft_prep, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, lamh, (cpx<float>*)K, lcomp,
                     nl, M);
  return hipGetLastError();
}

hipError_t launch_tfft_far(const void* ring, const void* K, void* far, int nl, long long n, int nx, int ny, int nz,
                           int kxs, hipStream_t s) {
  if (n % TF_S != 0 || nl < TF_S) return hipErrorInvalidValue;
  const Geo g{nx, ny, nz, kxs, nl};
  const long long ftot = (long long)(nz + 1) * (ny + 1) * (nx + 1);
  const long long nlog = (ftot + 31) / 32 * 4;
  if (nlog > (1LL << 30)) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)(((nlog + 7) / 8) * 8);
  hipLaunchKernelGGL(k_tfft_far, dim3(grid), dim3(192), 0, s, (const cpx<float>*)ring, (const cpx<float>*)K,
                     (cpx<float>*)far, g, n, tfft_blocks(nl), (int)nlog);
  return hipGetLastError();
}

}  // namespace motimpl
