// z pass of the circulant-embedded Green product (Eq. 11, Eq. 12): kernels
// and launchers, templated on the tile variant V.  Pencils
// along z for a kx tile at one ky, all components together, so that the
// 3x3 real spectral multiply sum_q Lambda_pq J_q sits between the forward and
// the inverse transform without leaving the workgroup; the fused pass takes
// ky and Py - ky in one workgroup, which share Lambda.
#pragma once

#include "fft_impl.h"

namespace motfft {

template <typename T, int M, int NC, bool INV, bool HIN, bool HOUT, int V>
__global__ __launch_bounds__((ZCfg<T, M, NC, V>::BLOCK)) void k_z_pass(
    const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, int kxn, int kxs, int ny, int rows_in, int rows_out,
    const cpx<T>* __restrict__ tw_g, int ntx, int nlog, Gate gate) {
  using C = ZCfg<T, M, NC, V>;
  constexpr int W = C::W, NP = C::NP, NPS = C::NPS;
  if (gate_closed(gate)) return;
  const int L = xcd_tile(blockIdx.x, nlog);
  if (L >= nlog) return;
  const int tile = L % ntx, ky = L / ntx;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = reinterpret_cast<cpx<T>*>(smem_raw + C::BUF);
  const int p = threadIdx.x % NP, jt = threadIdx.x / NP;
  const int comp = p / W, c = p - comp * W;
  const int kx = tile * W + c;
  const bool ok = kx < kxn;
  // the y-z buffer (yz_index) is the input of a forward pass and the output
  // of an inverse one; the other side is the full spectrum [comp][kz][ky][kxs]
  const size_t plane = (size_t)ny * kxs;
  const int kxc = ok ? kx : kxn - 1;
  const cpx<T>* src = INV ? in + ((size_t)comp * rows_in + jt) * plane + (size_t)ky * kxs + kxc
                          : in + yz_index(comp * rows_in + jt, ky, kxc, kxs, NC * rows_in);
  cpx<T>* dst = INV ? out + yz_index(comp * rows_out + jt, ky, kx, kxs, NC * rows_out)
                    : out + ((size_t)comp * rows_out + jt) * plane + (size_t)ky * kxs + kx;
  const size_t ss = INV ? plane : 16, ds = INV ? 16 : plane;
  cpx<T> v[PlanInfo<M>::E];
  load_first<T, M, HIN>(v, p, jt, [&](int, int, int u) { return src[(size_t)u * ss]; });
  load_table<cpx<T>, M, C::BLOCK>(tw, tw_g);
  run_fft<T, M, INV, HIN, HOUT, C::SPLIT>(v, lds, tw, p, jt, NPS, [&](int, int, int u, cpx<T> val) {
    if (ok) dst[(size_t)u * ds] = val;
  });
}

// Forward z FFT, Lambda multiply, inverse z FFT for the kx tile `tile` at
// ky = kyc and ky = ny - kyc (one row when kyc is 0 or ny/2).  Lambda is in
// the tile layout of lam_tile_offset: the workgroup's values form one
// contiguous range read for both ky rows.
//
// The multiply works in place on the spectra in LDS, one item (column c, kz)
// at a time for both ky rows, with the reflection signs of the compressed
// octant (xy odd in ky, xz odd in kz, yz odd in both).  Items are numbered
// with c fastest, so the Lambda words of a wave are contiguous; a thread's
// Lambda values are loaded when the kernel starts and arrive while the
// forward transform runs.
template <typename T, int M, int V>
__global__ __launch_bounds__((ZFCfg<T, M, V>::BLOCK)) void k_z_fused(
    const cpx<T>* in, cpx<T>* out, int kxn, int kxs, int ny, int rows_in, int rows_out,
    const T* __restrict__ lam, const cpx<T>* __restrict__ tw_g, int ntx, int nlog, Gate gate) {
  using C = ZFCfg<T, M, V>;
  constexpr int W = C::W, NP = C::NP, NPS = C::NPS, KZC = M / 2 + 1, BLOCK = C::BLOCK;
  constexpr int NI = W * M, KI = (NI + BLOCK - 1) / BLOCK;
  if (gate_closed(gate)) return;
  const int L = xcd_tile(blockIdx.x, nlog);
  if (L >= nlog) return;
  const int tile = L % ntx, kyc = L / ntx;
  const bool two = kyc != 0 && 2 * kyc != ny;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = lds + M * NPS;
  const int p = threadIdx.x % NP, jt = threadIdx.x / NP;
  const int h = p / (3 * W), q = (p / W) % 3, c = p % W;
  const int kx = tile * W + c;
  const bool okx = kx < kxn;
  const bool ok = okx && (h == 0 || two);
  const int ky = ok ? (h ? ny - kyc : kyc) : kyc;
  // both sides are the y-z buffer (yz_index): a z pencil has stride 16
  const cpx<T>* src = in + yz_index(q * rows_in + jt, ky, okx ? kx : kxn - 1, kxs, 3 * rows_in);
  cpx<T>* dst = out + yz_index(q * rows_out + jt, ky, kx, kxs, 3 * rows_out);
  cpx<T> v[PlanInfo<M>::E];
  load_first<T, M, true>(v, p, jt, [&](int, int, int u) { return src[(size_t)u * 16]; });
  // Lambda of this thread's items (component order xx, yy, zz, xy, xz, yz)
  const T* lt = lam + lam_tile_offset(tile * W, kyc, 0, 0, kxn, KZC, W);
  T lv[KI][6];
#pragma unroll
  for (int k = 0; k < KI; ++k) {
    const int it = (int)threadIdx.x + k * BLOCK;
    const int kz = it < NI ? it / W : 0, cc = it % W;
    const int kzc = kz <= M / 2 ? kz : M - kz;
#pragma unroll
    for (int comp = 0; comp < 6; ++comp) lv[k][comp] = lt[(kzc * W + cc) * 6 + comp];
  }
  load_table<cpx<T>, M, C::BLOCK>(tw, tw_g);
  run_fft<T, M, false, true, false>(v, lds, tw, p, jt, NPS,
                                    [&](int pp, int, int u, cpx<T> val) { lds[(jt + u) * NPS + pp] = val; });
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KI; ++k) {
    const int it = (int)threadIdx.x + k * BLOCK;
    if (KI * BLOCK > NI && it >= NI) break;
    const int kz = it / W, cc = it % W;
    const T sz = kz <= M / 2 ? (T)1 : (T)-1;
    const T lxx = lv[k][0], lyy = lv[k][1], lzz = lv[k][2];
    const T lxz = sz * lv[k][4];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      if (hh == 1 && !two) break;
      const T sy = hh ? (T)-1 : (T)1;
      const T lxy = sy * lv[k][3], lyz = sy * sz * lv[k][5];
      cpx<T>* r = lds + kz * NPS + hh * 3 * W + cc;
      const cpx<T> jx = r[0], jy = r[W], jz = r[2 * W];
      r[0] = cpx<T>{lxx * jx.x + lxy * jy.x + lxz * jz.x, lxx * jx.y + lxy * jy.y + lxz * jz.y};
      r[W] = cpx<T>{lxy * jx.x + lyy * jy.x + lyz * jz.x, lxy * jx.y + lyy * jy.y + lyz * jz.y};
      r[2 * W] = cpx<T>{lxz * jx.x + lyz * jy.x + lzz * jz.x, lxz * jx.y + lyz * jy.y + lzz * jz.y};
    }
  }
  __syncthreads();
  load_first<T, M, false>(v, p, jt, [&](int pp, int, int u) { return lds[(jt + u) * NPS + pp]; });
  __syncthreads();
  run_fft<T, M, true, false, true>(v, lds, tw, p, jt, NPS, [&](int, int, int u, cpx<T> val) {
    if (ok) dst[(size_t)u * 16] = val;
  });
}

template <typename T, int M, int NC, bool INV, bool HIN, bool HOUT, int V>
static hipError_t z_launch(const void* in, void* out, int kx, int kxs, int ny, int rows_in, int rows_out,
                           const void* tw, hipStream_t s, Gate g) {
  using C = ZCfg<T, M, NC, V>;
  const int ntx = (kx + C::W - 1) / C::W, nlog = ntx * ny;
  hipLaunchKernelGGL((k_z_pass<T, M, NC, INV, HIN, HOUT, V>), dim3(xcd_grid(nlog)), dim3(C::BLOCK), C::LDS, s,
                     (const cpx<T>*)in, (cpx<T>*)out, kx, kxs, ny, rows_in, rows_out, (const cpx<T>*)tw, ntx, nlog, g);
  return hipGetLastError();
}

template <typename T, int M, int V>
static hipError_t z_fused_launch(const void* in, void* out, int kx, int kxs, int ny, int rows_in, int rows_out,
                                 const T* lam, const void* tw, hipStream_t s, Gate g) {
  using C = ZFCfg<T, M, V>;
  const int ntx = (kx + C::W - 1) / C::W, nlog = ntx * (ny / 2 + 1);
  hipLaunchKernelGGL((k_z_fused<T, M, V>), dim3(xcd_grid(nlog)), dim3(C::BLOCK), C::LDS, s, (const cpx<T>*)in,
                     (cpx<T>*)out, kx, kxs, ny, rows_in, rows_out, lam, (const cpx<T>*)tw, ntx, nlog, g);
  return hipGetLastError();
}

// Supported forms: Z_FWD over 3 components with n_in = M/2, n_out = M
// (history), Z_FWD over 1 component with n_in = n_out = M (FP64 only, spectra
// precompute; tile variant 0 only), Z_INV over 3 components with n_in = M,
// n_out = M/2, and Z_FUSED over 3 components with n_in = n_out = M/2.
template <typename T, int V>
hipError_t z_pass_v(const void* in, void* out, int M, int mode, int nc, int kx, int kxs, int ny,
                    int rows_in, int n_in, int rows_out, int n_out, const T* lam, const void* tw,
                    hipStream_t s, Gate g) {
  if (n_in > rows_in || n_out > rows_out) return hipErrorInvalidValue;
  int form = -1;
  if (mode == Z_FWD && nc == 3 && 2 * n_in == M && n_out == M) form = 0;
  if (mode == Z_FWD && nc == 1 && n_in == M && n_out == M && sizeof(T) == 8 && V == 0) form = 1;
  if (mode == Z_INV && nc == 3 && n_in == M && 2 * n_out == M) form = 2;
  if (mode == Z_FUSED && nc == 3 && 2 * n_in == M && 2 * n_out == M && lam) form = 3;
  if (form < 0) return hipErrorInvalidValue;
  switch (M) {
#define X(m)                                                                                             \
  case m:                                                                                                \
    if (form == 0) return z_launch<T, m, 3, false, true, false, V>(in, out, kx, kxs, ny, rows_in, rows_out, tw, s, g); \
    if constexpr (sizeof(T) == 8 && V == 0)                                                              \
      if (form == 1) return z_launch<T, m, 1, false, false, false, V>(in, out, kx, kxs, ny, rows_in, rows_out, tw, s, g); \
    if (form == 2) return z_launch<T, m, 3, true, false, true, V>(in, out, kx, kxs, ny, rows_in, rows_out, tw, s, g); \
    return z_fused_launch<T, m, V>(in, out, kx, kxs, ny, rows_in, rows_out, lam, tw, s, g);
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// Explicit instantiations of one tile variant (each variant has its own
// translation unit so that they compile in parallel).
#define MOT_Z_VARIANT(V)                                                                                       \
  template hipError_t z_pass_v<float, V>(const void*, void*, int, int, int, int, int, int, int, int, int, int, \
                                         const float*, const void*, hipStream_t, Gate);                        \
  template hipError_t z_pass_v<double, V>(const void*, void*, int, int, int, int, int, int, int, int, int,     \
                                          int, const double*, const void*, hipStream_t, Gate);

}  // namespace motfft
