// y pass of the circulant-embedded Green product (Eq. 11): kernels and
// launchers, templated on the tile variant V.  Complex pencils
// along y for a tile of kx columns.  The forward pass of a product reads only
// the Ny physical rows (the rest of the doubled grid is zero), the inverse
// writes only the Ny rows that the truncation back to the physical grid keeps.
#pragma once

#include "fft_impl.h"

namespace motfft {

template <typename T, int M, bool INV, bool HIN, bool HOUT, int V>
__global__ __launch_bounds__((YCfg<T, M, V>::BLOCK)) void k_y_pass(const cpx<T>* __restrict__ in,
                                                               cpx<T>* __restrict__ out, int kxn, int kxs,
                                                               int rows_in, int rows_out,
                                                               const cpx<T>* __restrict__ tw_g, int ntx, int nlog,
                                                               Gate gate) {
  using C = YCfg<T, M, V>;
  constexpr int NP = C::NP, NPS = C::NPS;
  if (gate_closed(gate)) return;
  const int L = xcd_tile(blockIdx.x, nlog);
  if (L >= nlog) return;
  const int tile = L % ntx, plane = L / ntx;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* twl = reinterpret_cast<cpx<T>*>(smem_raw + C::BUF);
  const cpx<T>* tw = C::TWG ? tw_g : twl;
  const int p = threadIdx.x % NP, jt = threadIdx.x / NP;
  const int kx = tile * NP + p;
  const bool ok = kx < kxn;
  // columns past the last kx load a valid column and store nothing; the
  // complex side (output of the forward pass, input of the inverse) is the
  // y-z buffer (yz_index) of nlog / ntx planes
  const int kxc = ok ? kx : kxn - 1;
  const int P = nlog / ntx;
  const size_t RS = yz_row_stride(kxs, P);
  const cpx<T>* src = INV ? in + yz_index(plane, jt, kxc, kxs, P) : in + ((size_t)plane * rows_in + jt) * kxs + kxc;
  cpx<T>* dst = INV ? out + ((size_t)plane * rows_out + jt) * kxs + kx : out + yz_index(plane, jt, kx, kxs, P);
  const size_t ss = INV ? RS : (size_t)kxs, ds = INV ? (size_t)kxs : RS;
  // the y-z buffer is produced once and read once per product: past 32 MB
  // the forward pass writes it and the inverse pass reads it with streaming
  // (nontemporal) accesses, so that it does not evict the lines the next
  // pass reads (the x inverse pass's input, which the inverse pass writes);
  // only by tiles whose columns fill whole 128-byte lines (narrower streaming
  // accesses reach HBM as partial lines)
  constexpr bool NT_TILE = C::NP * sizeof(cpx<T>) >= 128;
  const bool big = NT_TILE && (size_t)M * RS * sizeof(cpx<T>) >= ((size_t)32 << 20);
  typedef T tv2 __attribute__((ext_vector_type(2)));
  cpx<T> v[PlanInfo<M>::E];
  load_first<T, M, HIN>(v, p, jt, [&](int, int, int u) {
    const cpx<T>* q = src + (size_t)u * ss;
    if constexpr (INV) {
      if (big) {
        const tv2 t = __builtin_nontemporal_load(reinterpret_cast<const tv2*>(q));
        return cpx<T>{t.x, t.y};
      }
    }
    return *q;
  });
  // the twiddles are first read after the first exchange's barrier
  if constexpr (!C::TWG) load_table<cpx<T>, M, C::BLOCK>(twl, tw_g);
  run_fft<T, M, INV, HIN, HOUT, C::SPLIT>(v, lds, tw, p, jt, NPS, [&](int, int, int u, cpx<T> val) {
    if (!ok) return;
    cpx<T>* q = dst + (size_t)u * ds;
    if constexpr (!INV) {
      if (big) {
        const tv2 t = {val.x, val.y};
        __builtin_nontemporal_store(t, reinterpret_cast<tv2*>(q));
        return;
      }
    }
    *q = val;
  });
}

template <typename T, int M, bool INV, bool HIN, bool HOUT, int V>
static hipError_t y_launch(const void* in, void* out, int kx, int kxs, int planes, int rows_in, int rows_out,
                           const void* tw, hipStream_t s, Gate g) {
  using C = YCfg<T, M, V>;
  const int ntx = (kx + C::NP - 1) / C::NP, nlog = ntx * planes;
  hipLaunchKernelGGL((k_y_pass<T, M, INV, HIN, HOUT, V>), dim3(xcd_grid(nlog)), dim3(C::BLOCK), C::LDS, s,
                     (const cpx<T>*)in, (cpx<T>*)out, kx, kxs, rows_in, rows_out, (const cpx<T>*)tw, ntx, nlog, g);
  return hipGetLastError();
}

// Supported forms: forward with n_in = M/2 (product) or M (FP64 only,
// spectra precompute; tile variant 0 only), both with n_out = M; inverse with
// n_in = M, n_out = M/2.
template <typename T, int V>
hipError_t y_pass_v(const void* in, void* out, int M, bool inverse, int kx, int kxs, int planes,
                    int rows_in, int n_in, int rows_out, int n_out, const void* tw, hipStream_t s, Gate g) {
  if (n_in > rows_in || n_out > rows_out) return hipErrorInvalidValue;
  const int form = !inverse && 2 * n_in == M && n_out == M   ? 0
                   : !inverse && n_in == M && n_out == M       ? 1
                   : inverse && n_in == M && 2 * n_out == M    ? 2
                                                               : -1;
  if (form < 0 || (form == 1 && (sizeof(T) != 8 || V != 0))) return hipErrorInvalidValue;
  switch (M) {
#define X(m)                                                                                     \
  case m:                                                                                        \
    if (form == 0) return y_launch<T, m, false, true, false, V>(in, out, kx, kxs, planes, rows_in, rows_out, tw, s, g); \
    if constexpr (sizeof(T) == 8 && V == 0)                                                      \
      if (form == 1)                                                                             \
        return y_launch<T, m, false, false, false, V>(in, out, kx, kxs, planes, rows_in, rows_out, tw, s, g);        \
    return y_launch<T, m, true, false, true, V>(in, out, kx, kxs, planes, rows_in, rows_out, tw, s, g);
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// Explicit instantiations of one tile variant (each variant has its own
// translation unit so that they compile in parallel).
#define MOT_Y_VARIANT(V)                                                                                      \
  template hipError_t y_pass_v<float, V>(const void*, void*, int, bool, int, int, int, int, int, int, int,    \
                                         const void*, hipStream_t, Gate);                                     \
  template hipError_t y_pass_v<double, V>(const void*, void*, int, bool, int, int, int, int, int, int, int,   \
                                          const void*, hipStream_t, Gate);

}  // namespace motfft
