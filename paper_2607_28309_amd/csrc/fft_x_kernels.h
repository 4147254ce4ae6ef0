// x pass of the circulant-embedded Green product (Eq. 11, Eq. 12): kernels
// and launchers, templated on the tile variant V.
//
// Forward: a real row of length 2M (zero beyond the first n_in pairs) is
//   packed as z[n] = x[2n] + i x[2n+1], transformed with a length-M complex
//   FFT and unpacked to the M+1 non-redundant bins
//   X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) W_{2M}^k (Z[k] - conj Z[M-k]).
// Inverse: Z[k] = (X[k] + conj X[M-k]) + i W_{2M}^{-k} (X[k] - conj X[M-k]),
//   the inverse length-M FFT, and the first M/2 pairs (the physical row) go
//   straight from registers into the diagonal terms of Eq. 12.
//
// Lanes walk along a row (jt fastest), so row loads and stores are coalesced.
#pragma once

#include "fft_impl.h"

namespace motfft {

// Row of local slot p in this workgroup.  With 3 components a workgroup
// takes G = NP/3 voxel rows in all three components, so the (per-voxel)
// permittivity row read by the epilogue is fetched from HBM once; returns
// nrows (invalid) for slots beyond the data.
template <int NP>
__device__ __forceinline__ int xrow(int p, int ncomp, int rows_per_comp, int nrows) {
  if (ncomp == 3 && NP >= 3) {
    constexpr int G = NP / 3 > 0 ? NP / 3 : 1;
    if (p >= 3 * G) return nrows;
    const int comp = p / G, vr = blockIdx.x * G + (p - comp * G);
    return vr < rows_per_comp ? comp * rows_per_comp + vr : nrows;
  }
  const int r = blockIdx.x * NP + p;
  return r < nrows ? r : nrows;
}

// pre (optional, per voxel row like the epilogue's permittivity): the input
// is multiplied by (pre - 1) as it is loaded, i.e. the contrast applied on the
// input for the transposed operators.
template <typename T, typename IO, int M, bool HIN, int V>
__global__ __launch_bounds__((XCfg<T, M, V>::BLOCK)) void k_x_forward(const IO* __restrict__ in,
                                                                  cpx<T>* __restrict__ out, int nrows,
                                                                  int rows_per_comp, int ncomp, int row_len,
                                                                  int kxs, const cpx<T>* __restrict__ tw_g,
                                                                  const cpx<T>* __restrict__ tw2_g,
                                                                  const double* __restrict__ pre, Gate gate) {
  using C = XCfg<T, M, V>;
  constexpr int NP = C::NP, NPS = C::NPS, TJ = C::TJ, E = PlanInfo<M>::E;
  if (gate_closed(gate)) return;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = lds + (M + 1) * NPS;
  cpx<T>* tw2 = tw + M;
  using V2 = typename io2<IO>::t;
  const int jt = threadIdx.x % TJ, p = threadIdx.x / TJ;
  const int grow = xrow<NP>(p, ncomp, rows_per_comp, nrows);
  const bool valid = grow < nrows;
  const IO* src = in + (size_t)(valid ? grow : 0) * row_len + 2 * jt;
  const double* prow = pre ? pre + (size_t)((valid ? grow : 0) % rows_per_comp) * row_len + 2 * jt : nullptr;
  cpx<T> v[E];
  load_first<T, M, HIN>(v, p, jt, [&](int, int, int u) {
    const V2 pr = *reinterpret_cast<const V2*>(src + 2 * u);
    if (prow) {
      const double2 x2 = *reinterpret_cast<const double2*>(prow + 2 * u);
      return cpx<T>{(T)((double)pr.x * (x2.x - 1.0)), (T)((double)pr.y * (x2.y - 1.0))};
    }
    return cpx<T>{(T)pr.x, (T)pr.y};
  });
  load_table<cpx<T>, M, C::BLOCK>(tw, tw_g);
  load_table<cpx<T>, M + 1, C::BLOCK>(tw2, tw2_g);
  run_fft<T, M, false, HIN, false>(v, lds, tw, p, jt, NPS,
                                   [&](int pp, int, int u, cpx<T> val) { lds[(jt + u) * NPS + pp] = val; });
  __syncthreads();
  if (!valid) return;
  // bins k = jt + TJ i of row p (and k = M by lane jt = 0)
  cpx<T>* dst = out + (size_t)grow * kxs + jt;
  const cpx<T>* zr = lds + p;
  auto unpack = [&](cpx<T> zk, cpx<T> zm, cpx<T> w) {
    // E = (zk + conj zm)/2, O = -i/2 (zk - conj zm), X = E + w O
    const cpx<T> ev{(T)0.5 * (zk.x + zm.x), (T)0.5 * (zk.y - zm.y)};
    const cpx<T> od{(T)0.5 * (zk.y + zm.y), (T)-0.5 * (zk.x - zm.x)};
    return cadd(ev, cmul(w, od));
  };
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = jt + TJ * i;
    const int m = i == 0 ? (jt == 0 ? 0 : M - jt) : M - k;
    dst[TJ * i] = unpack(zr[k * NPS], zr[m * NPS], tw2[k]);
  }
  if (jt == 0) dst[M] = unpack(zr[0], zr[0], tw2[M]);
}

template <typename T, typename IO, int M, int V>
__global__ __launch_bounds__((XCfg<T, M, V>::BLOCK)) void k_x_inverse(
    const cpx<T>* __restrict__ in, IO* __restrict__ y, const IO* __restrict__ J,
    const double* __restrict__ eps, Epilogue ep, int nrows, int rows_per_comp, int ncomp, int row_len,
    int kxs, const cpx<T>* __restrict__ tw_g, const cpx<T>* __restrict__ tw2_g, Gate gate) {
  using C = XCfg<T, M, V>;
  constexpr int NP = C::NP, NPS = C::NPS, TJ = C::TJ, E = PlanInfo<M>::E;
  if (gate_closed(gate)) return;
  static_assert((M / 2) % TJ == 0, "the kept half of a row is whole columns of the lane layout");
  constexpr int EH = E / 2;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = lds + (M + 1) * NPS;
  cpx<T>* tw2 = tw + M;
  using V2 = typename io2<IO>::t;
  const int jt = threadIdx.x % TJ, p = threadIdx.x / TJ;
  const int grow = xrow<NP>(p, ncomp, rows_per_comp, nrows);
  const bool valid = grow < nrows;
  const int growc = valid ? grow : 0;
  // bins k = jt + TJ i and k = M of row p, all loads issued before any wait
  const cpx<T>* srow = in + (size_t)growc * kxs;
  cpx<T> x[E];
#pragma unroll
  for (int i = 0; i < E; ++i) x[i] = srow[jt + TJ * i];
  const cpx<T> xM = srow[M];
  // epilogue operands of the pairs n = jt + TJ i (i < E/2) this lane writes
  const size_t roff = (size_t)growc * row_len + 2 * jt;
  const size_t eoff = (size_t)(growc % rows_per_comp) * row_len + 2 * jt;
  V2 jv[EH];
  double2 ev[EH];
#pragma unroll
  for (int i = 0; i < EH; ++i) {
    jv[i] = *reinterpret_cast<const V2*>(J + roff + 2 * TJ * i);
    ev[i] = *reinterpret_cast<const double2*>(eps + eoff + 2 * TJ * i);
  }
  load_table<cpx<T>, M, C::BLOCK>(tw, tw_g);
  load_table<cpx<T>, M + 1, C::BLOCK>(tw2, tw2_g);
  cpx<T>* xr = lds + p;
#pragma unroll
  for (int i = 0; i < E; ++i) xr[(jt + TJ * i) * NPS] = x[i];
  if (jt == 0) xr[M * NPS] = xM;
  __syncthreads();
  cpx<T> v[E];
  load_first<T, M, false>(v, p, jt, [&](int, int, int u) {
    const int k = jt + u;
    const cpx<T> xk = xr[k * NPS], xm = xr[(M - k) * NPS];
    // Z[k] = (Xk + conj Xm) + i W^{-k} (Xk - conj Xm)
    const cpx<T> dk{xk.x - xm.x, xk.y + xm.y};
    const cpx<T> rk = cmulc(dk, tw2[k]);
    return cpx<T>{xk.x + xm.x - rk.y, xk.y - xm.y + rk.x};
  });
  __syncthreads();
  IO* yrow = y + roff;
  run_fft<T, M, true, false, true>(v, lds, tw, p, jt, NPS, [&](int, int, int u, cpx<T> z) {
    if (!valid) return;
    const int i = u / TJ;
    const double2 e2 = ev[i];
    const V2 j2 = jv[i];
    V2 r;
    r.x = (IO)(((T)(ep.ca * e2.x + ep.c0)) * (T)j2.x + ((T)(ep.cb * e2.x + ep.cb0)) * z.x);
    r.y = (IO)(((T)(ep.ca * e2.y + ep.c0)) * (T)j2.y + ((T)(ep.cb * e2.y + ep.cb0)) * z.y);
    *reinterpret_cast<V2*>(yrow + 2 * u) = r;
  });
}

template <int NP>
static int x_blocks(int nrows, int rows_per_comp, int ncomp) {
  return (ncomp == 3 && NP >= 3) ? (rows_per_comp + NP / 3 - 1) / (NP / 3) : (nrows + NP - 1) / NP;
}

// Supported forms: n_in = M/2 (product: rows of M reals) or n_in = M (FP64
// only, spectra precompute: rows of 2M reals; tile variant 0 only).
template <typename T, typename IO, int V>
hipError_t x_forward_v(const IO* in, void* out, int M, int nrows, int rows_per_comp, int ncomp, int row_len,
                       int n_in, int kxs, const void* tw, const void* tw2, hipStream_t s, const double* pre,
                       Gate gg) {
  const bool half = 2 * n_in == M;
  if ((!half && n_in != M) || (!half && (sizeof(T) != 8 || V != 0)) || 2 * n_in > row_len || kxs < M + 1 ||
      (pre && !half))
    return hipErrorInvalidValue;
  switch (M) {
#define X(m)                                                                                              \
  case m: {                                                                                               \
    using C = XCfg<T, m, V>;                                                                              \
    const dim3 g(x_blocks<C::NP>(nrows, rows_per_comp, ncomp));                                           \
    if (half)                                                                                             \
      hipLaunchKernelGGL((k_x_forward<T, IO, m, true, V>), g, dim3(C::BLOCK), C::LDS, s, in, (cpx<T>*)out, \
                         nrows, rows_per_comp, ncomp, row_len, kxs, (const cpx<T>*)tw, (const cpx<T>*)tw2, pre, gg); \
    else if constexpr (sizeof(T) == 8 && sizeof(IO) == 8 && V == 0)                                      \
      hipLaunchKernelGGL((k_x_forward<T, IO, m, false, V>), g, dim3(C::BLOCK), C::LDS, s, in, (cpx<T>*)out, \
                         nrows, rows_per_comp, ncomp, row_len, kxs, (const cpx<T>*)tw, (const cpx<T>*)tw2, nullptr, gg); \
    return hipGetLastError();                                                                             \
  }
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// Supported form: n_out = M reals (the physical half of the length-2M row).
template <typename T, typename IO, int V>
hipError_t x_inverse_v(const void* in, IO* y, const IO* J, const double* eps, Epilogue ep, int M, int nrows,
                       int rows_per_comp, int ncomp, int row_len, int n_out, int kxs, const void* tw,
                       const void* tw2, hipStream_t s, Gate gg) {
  if (n_out != M || row_len < M || kxs < M + 1) return hipErrorInvalidValue;
  switch (M) {
#define X(m)                                                                                            \
  case m: {                                                                                             \
    using C = XCfg<T, m, V>;                                                                            \
    const dim3 g(x_blocks<C::NP>(nrows, rows_per_comp, ncomp));                                         \
    hipLaunchKernelGGL((k_x_inverse<T, IO, m, V>), g, dim3(C::BLOCK), C::LDS, s, (const cpx<T>*)in, y, J, eps, \
                       ep, nrows, rows_per_comp, ncomp, row_len, kxs, (const cpx<T>*)tw, (const cpx<T>*)tw2, gg); \
    return hipGetLastError();                                                                           \
  }
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// Explicit instantiations of one tile variant (each variant has its own
// translation unit so that they compile in parallel).
#define MOT_X_VARIANT(V)                                                                                       \
  MOT_X_VARIANT_T(float, float, V)                                                                             \
  MOT_X_VARIANT_T(float, double, V)                                                                            \
  MOT_X_VARIANT_T(double, double, V)
#define MOT_X_VARIANT_T(T, IO, V)                                                                              \
  template hipError_t x_forward_v<T, IO, V>(const IO*, void*, int, int, int, int, int, int, int, const void*,  \
                                            const void*, hipStream_t, const double*, Gate);                    \
  template hipError_t x_inverse_v<T, IO, V>(const void*, IO*, const IO*, const double*, Epilogue, int, int,    \
                                            int, int, int, int, int, const void*, const void*, hipStream_t, Gate);

}  // namespace motfft
