// FFT passes of the circulant-embedded Green product (Eq. 11, Eq. 12).
//
// x pass: a real row of length 2M (zero beyond the first n_in pairs) is
//   packed as z[n] = x[2n] + i x[2n+1], transformed with a length-M complex
//   FFT and unpacked to the M+1 non-redundant bins
//   X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) W_{2M}^k (Z[k] - conj Z[M-k]).
//   The inverse repacks Z[k] = (X[k] + conj X[M-k]) + i W_{2M}^{-k} (X[k] - conj X[M-k]),
//   applies the inverse length-M FFT and keeps the first n_out reals, fused
//   with the diagonal terms of Eq. 12.
// y pass: complex pencils along y for a tile of kx columns; the forward pass
//   reads only the Ny physical rows (the rest of the doubled grid is zero),
//   the inverse writes only the Ny rows that the truncation T{} keeps.
// z pass: pencils along z for a kx tile at one ky, all components together,
//   so that the 3x3 real spectral multiply sum_q Lambda_pq J_q sits between
//   the forward and the inverse transform without leaving the workgroup; the
//   fused pass takes ky and Py - ky in one workgroup, which share Lambda.
//
// Workgroups of the y and z passes are issued in an XCD-aware order: the
// hardware hands consecutive workgroup ids to the eight XCDs in turn, each
// with its own L2, so logical tile t is given to id (t mod Q) * 8 + t / Q
// (Q = ceil(tiles/8)); neighbouring kx tiles of one row then share an L2 and
// the 128-byte lines they split are fetched from HBM once.
#include "fft_core.h"
#include "fft_passes.h"

namespace motfft {

constexpr int floor_pow2(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int LDS_BUDGET = 81920;

// LDS rows are padded to NPS = NP + 1 entries so that lanes walking along a
// pencil (stride NPS) and the row stride of the Stockham writes spread over
// the LDS banks instead of hitting the same ones.
template <typename T, int M> struct XCfg {
  static constexpr int TJ = PlanInfo<M>::TJ;
  static constexpr int SZ = (int)sizeof(cpx<T>);
  static constexpr int NP =
      cmax(1, floor_pow2(cmin(256 / TJ, (LDS_BUDGET - (2 * M + 1) * SZ) / ((M + 1) * SZ) - 1)));
  static constexpr int NPS = NP + 1;
  static constexpr int BLOCK = NP * TJ;
  static constexpr size_t LDS = (size_t)((M + 1) * NPS + 2 * M + 1) * SZ;
};
template <typename T, int M> struct YCfg {
  static constexpr int TJ = PlanInfo<M>::TJ;
  static constexpr int SZ = (int)sizeof(cpx<T>);
  static constexpr int NP = cmax(1, floor_pow2(cmin(cmin(256 / TJ, 32), (LDS_BUDGET - M * SZ) / (M * SZ) - 1)));
  static constexpr int NPS = NP + 1;
  static constexpr int BLOCK = NP * TJ;
  static constexpr size_t LDS = (size_t)(M * NPS + M) * SZ;
};
template <typename T, int M, int NC> struct ZCfg {
  static constexpr int TJ = PlanInfo<M>::TJ;
  static constexpr int SZ = (int)sizeof(cpx<T>);
  static constexpr int W =
      cmax(1, floor_pow2(cmin(cmin(16, 1024 / (NC * TJ)), (LDS_BUDGET - 2 * M * SZ) / (NC * M * SZ))));
  static constexpr int NP = NC * W;
  static constexpr int NPS = NP + 1;
  static constexpr int BLOCK = NP * TJ;
  static constexpr size_t LDS = (size_t)(M * NPS + M) * SZ;
};

// z pass with the spectral multiply: W kx columns x 3 components x 2 ky rows.
template <typename T, int M> struct ZFCfg {
  static constexpr int TJ = PlanInfo<M>::TJ;
  static constexpr int SZ = (int)sizeof(cpx<T>);
  static constexpr int W =
      cmax(1, floor_pow2(cmin(cmin(16, 1024 / (6 * TJ)), (LDS_BUDGET - 2 * M * SZ) / (6 * M * SZ))));
  static constexpr int NP = 6 * W;
  static constexpr int NPS = NP + 1;
  static constexpr int BLOCK = NP * TJ;
  static constexpr size_t LDS = (size_t)(M * NPS + M) * SZ;
};

constexpr int NXCD = 8;
// logical tile of workgroup id b; tiles >= nlog are idle
__device__ __forceinline__ int xcd_tile(int b, int nlog) {
  const int q = (nlog + NXCD - 1) / NXCD;
  return (b % NXCD) * q + b / NXCD;
}
inline int xcd_grid(int nlog) { return ((nlog + NXCD - 1) / NXCD) * NXCD; }

template <typename T, int M>
__device__ __forceinline__ void load_table(cpx<T>* dst, const cpx<T>* src, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

template <typename IO> struct io2;
template <> struct io2<float> { using t = float2; };
template <> struct io2<double> { using t = double2; };

// ------------------------------------------------------------------ x pass
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

template <typename T, typename IO, int M>
__global__ __launch_bounds__((XCfg<T, M>::BLOCK)) void k_x_forward(const IO* __restrict__ in,
                                                                  cpx<T>* __restrict__ out, int nrows,
                                                                  int rows_per_comp, int ncomp, int row_len,
                                                                  int n_in, int kxs,
                                                                  const cpx<T>* __restrict__ tw_g,
                                                                  const cpx<T>* __restrict__ tw2_g) {
  using C = XCfg<T, M>;
  constexpr int NP = C::NP, NPS = C::NPS;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = lds + (M + 1) * NPS;
  cpx<T>* tw2 = tw + M;
  load_table<T, M>(tw, tw_g, M);
  load_table<T, M>(tw2, tw2_g, M + 1);
  using V2 = typename io2<IO>::t;
  __syncthreads();
  // lanes walk along a row (jt fastest): the first stage loads its inputs
  // straight from the contiguous row, 2 reals per complex element
  const int jt = threadIdx.x % C::TJ, p = threadIdx.x / C::TJ;
  const int grow_p = xrow<NP>(p, ncomp, rows_per_comp, nrows);
  const IO* src = in + (size_t)grow_p * row_len;
  cpx<T> v[PlanInfo<M>::E];
  load_first<T, M>(v, p, jt, [&](int, int e) {
    if (grow_p < nrows && e < n_in) {
      const V2 pr = *reinterpret_cast<const V2*>(src + 2 * e);
      return cpx<T>{(T)pr.x, (T)pr.y};
    }
    return cpx<T>{(T)0, (T)0};
  });
  run_fft<T, M, false>(v, lds, tw, p, jt, NPS, [&](int pp, int e, cpx<T> val) { lds[e * NPS + pp] = val; });
  __syncthreads();
  for (int idx = threadIdx.x; idx < NP * (M + 1); idx += blockDim.x) {
    const int row = idx / (M + 1), k = idx - row * (M + 1);
    const int grow = xrow<NP>(row, ncomp, rows_per_comp, nrows);
    if (grow >= nrows) continue;
    const cpx<T> zk = lds[(k == M ? 0 : k) * NPS + row];
    const cpx<T> zm = lds[(k == 0 ? 0 : M - k) * NPS + row];
    // E = (zk + conj zm)/2, O = -i/2 (zk - conj zm)
    const cpx<T> e{(T)0.5 * (zk.x + zm.x), (T)0.5 * (zk.y - zm.y)};
    const cpx<T> o{(T)0.5 * (zk.y + zm.y), (T)-0.5 * (zk.x - zm.x)};
    out[(size_t)grow * kxs + k] = cadd(e, cmul(tw2[k], o));
  }
}

template <typename T, typename IO, int M>
__global__ __launch_bounds__((XCfg<T, M>::BLOCK)) void k_x_inverse(
    const cpx<T>* __restrict__ in, IO* __restrict__ y, const IO* __restrict__ J,
    const double* __restrict__ eps, Epilogue ep, int nrows, int rows_per_comp, int ncomp, int row_len,
    int n_out, int kxs, const cpx<T>* __restrict__ tw_g, const cpx<T>* __restrict__ tw2_g) {
  using C = XCfg<T, M>;
  constexpr int NP = C::NP, NPS = C::NPS;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = lds + (M + 1) * NPS;
  cpx<T>* tw2 = tw + M;
  load_table<T, M>(tw, tw_g, M);
  load_table<T, M>(tw2, tw2_g, M + 1);
  for (int idx = threadIdx.x; idx < NP * (M + 1); idx += blockDim.x) {
    const int row = idx / (M + 1), k = idx - row * (M + 1);
    const int grow = xrow<NP>(row, ncomp, rows_per_comp, nrows);
    lds[k * NPS + row] = grow < nrows ? in[(size_t)grow * kxs + k] : cpx<T>{(T)0, (T)0};
  }
  __syncthreads();
  constexpr int H = M / 2 + 1;
  for (int idx = threadIdx.x; idx < NP * H; idx += blockDim.x) {
    const int row = idx / H, k = idx - row * H;
    const int m = M - k;
    const cpx<T> xk = lds[k * NPS + row];
    const cpx<T> xm = lds[m * NPS + row];
    // Z[k] = (Xk + conj Xm) + i W^{-k} (Xk - conj Xm)
    const cpx<T> dk{xk.x - xm.x, xk.y + xm.y};
    const cpx<T> rk = cmulc(dk, tw2[k]);
    const cpx<T> zk{xk.x + xm.x - rk.y, xk.y - xm.y + rk.x};
    const cpx<T> dm{xm.x - xk.x, xm.y + xk.y};
    const cpx<T> rm = cmulc(dm, tw2[m]);
    const cpx<T> zm{xm.x + xk.x - rm.y, xm.y - xk.y + rm.x};
    lds[k * NPS + row] = zk;
    if (m < M && m != k) lds[m * NPS + row] = zm;
  }
  __syncthreads();
  const int jt = threadIdx.x % C::TJ, p = threadIdx.x / C::TJ;
  cpx<T> v[PlanInfo<M>::E];
  load_first<T, M>(v, p, jt, [&](int pp, int e) { return lds[e * NPS + pp]; });
  __syncthreads();
  // the last stage hands z[n] = (x[2n], x[2n+1]) to the epilogue directly
  using V2 = typename io2<IO>::t;
  const int grow_p = xrow<NP>(p, ncomp, rows_per_comp, nrows);
  const int half = n_out / 2;
  const size_t roff = (size_t)grow_p * row_len;
  const size_t eoff0 = (size_t)(grow_p % rows_per_comp) * row_len;
  run_fft<T, M, true>(v, lds, tw, p, jt, NPS, [&](int, int n, cpx<T> z) {
    if (grow_p >= nrows || n >= half) return;
    const size_t off = roff + 2 * n;
    const double2 e2 = *reinterpret_cast<const double2*>(eps + eoff0 + 2 * n);
    const V2 j2 = *reinterpret_cast<const V2*>(J + off);
    V2 r;
    r.x = (IO)(((T)(ep.ca * e2.x + ep.c0)) * (T)j2.x + ((T)(ep.cb * e2.x + ep.cb0)) * z.x);
    r.y = (IO)(((T)(ep.ca * e2.y + ep.c0)) * (T)j2.y + ((T)(ep.cb * e2.y + ep.cb0)) * z.y);
    *reinterpret_cast<V2*>(y + off) = r;
  });
}

// ------------------------------------------------------------------ y pass
template <typename T, int M, bool INV>
__global__ __launch_bounds__((YCfg<T, M>::BLOCK)) void k_y_pass(const cpx<T>* __restrict__ in,
                                                               cpx<T>* __restrict__ out, int kxn, int kxs,
                                                               int rows_in, int n_in, int rows_out,
                                                               int n_out, const cpx<T>* __restrict__ tw_g,
                                                               int ntx, int nlog) {
  using C = YCfg<T, M>;
  constexpr int NP = C::NP, NPS = C::NPS;
  const int L = xcd_tile(blockIdx.x, nlog);
  if (L >= nlog) return;
  const int tile = L % ntx, plane = L / ntx;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = lds + M * NPS;
  load_table<T, M>(tw, tw_g, M);
  __syncthreads();
  const int p = threadIdx.x % NP, jt = threadIdx.x / NP;
  const int kx = tile * NP + p;
  const bool ok = kx < kxn;
  const cpx<T>* src = in + (size_t)plane * rows_in * kxs + kx;
  cpx<T>* dst = out + (size_t)plane * rows_out * kxs + kx;
  cpx<T> v[PlanInfo<M>::E];
  load_first<T, M>(v, p, jt, [&](int, int e) {
    return (ok && e < n_in) ? src[(size_t)e * kxs] : cpx<T>{(T)0, (T)0};
  });
  run_fft<T, M, INV>(v, lds, tw, p, jt, NPS, [&](int, int e, cpx<T> val) {
    if (ok && e < n_out) dst[(size_t)e * kxs] = val;
  });
}

// ------------------------------------------------------------------ z pass
template <typename T, int M, int NC, bool INV>
__global__ __launch_bounds__((ZCfg<T, M, NC>::BLOCK)) void k_z_pass(
    const cpx<T>* __restrict__ in, cpx<T>* __restrict__ out, int kxn, int kxs, int ny, int rows_in, int n_in,
    int rows_out, int n_out, const cpx<T>* __restrict__ tw_g, int ntx, int nlog) {
  using C = ZCfg<T, M, NC>;
  constexpr int W = C::W, NP = C::NP, NPS = C::NPS;
  const int L = xcd_tile(blockIdx.x, nlog);
  if (L >= nlog) return;
  const int tile = L % ntx, ky = L / ntx;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = lds + M * NPS;
  load_table<T, M>(tw, tw_g, M);
  __syncthreads();
  const int p = threadIdx.x % NP, jt = threadIdx.x / NP;
  const int comp = p / W, c = p - comp * W;
  const int kx = tile * W + c;
  const bool ok = kx < kxn;
  const size_t plane = (size_t)ny * kxs;
  const cpx<T>* src = in + ((size_t)comp * rows_in) * plane + (size_t)ky * kxs + kx;
  cpx<T>* dst = out + ((size_t)comp * rows_out) * plane + (size_t)ky * kxs + kx;
  cpx<T> v[PlanInfo<M>::E];
  load_first<T, M>(v, p, jt, [&](int, int e) {
    return (ok && e < n_in) ? src[(size_t)e * plane] : cpx<T>{(T)0, (T)0};
  });
  run_fft<T, M, INV>(v, lds, tw, p, jt, NPS, [&](int, int e, cpx<T> val) {
    if (ok && e < n_out) dst[(size_t)e * plane] = val;
  });
}

// Forward z FFT, Lambda multiply, inverse z FFT for the kx tile `tile` at
// ky = kyc and ky = ny - kyc (one row when kyc is 0 or ny/2).  Lambda is in
// the tile layout [kyc][kx][kzc][6] (kx < kxn): the workgroup's values form
// one contiguous range read once for both ky rows.
template <typename T, int M>
__global__ __launch_bounds__((ZFCfg<T, M>::BLOCK)) void k_z_fused(
    const cpx<T>* in, cpx<T>* out, int kxn, int kxs, int ny, int rows_in, int n_in, int rows_out, int n_out,
    const T* __restrict__ lam, const cpx<T>* __restrict__ tw_g, int ntx, int nlog) {
  using C = ZFCfg<T, M>;
  constexpr int W = C::W, NP = C::NP, NPS = C::NPS, KZC = M / 2 + 1;
  const int L = xcd_tile(blockIdx.x, nlog);
  if (L >= nlog) return;
  const int tile = L % ntx, kyc = L / ntx;
  const bool two = kyc != 0 && 2 * kyc != ny;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = lds + M * NPS;
  load_table<T, M>(tw, tw_g, M);
  __syncthreads();
  const int p = threadIdx.x % NP, jt = threadIdx.x / NP;
  const int h = p / (3 * W), comp = (p / W) % 3, c = p % W;
  const int kx0 = tile * W;
  const int kx = kx0 + c;
  const int ky = h ? ny - kyc : kyc;
  const bool ok = kx < kxn && (h == 0 || two);
  const size_t plane = (size_t)ny * kxs;
  const cpx<T>* src = in + ((size_t)comp * rows_in) * plane + (size_t)ky * kxs + kx;
  cpx<T>* dst = out + ((size_t)comp * rows_out) * plane + (size_t)ky * kxs + kx;
  cpx<T> v[PlanInfo<M>::E];
  load_first<T, M>(v, p, jt, [&](int, int e) {
    return (ok && e < n_in) ? src[(size_t)e * plane] : cpx<T>{(T)0, (T)0};
  });
  run_fft<T, M, false>(v, lds, tw, p, jt, NPS, [&](int pp, int e, cpx<T> val) { lds[e * NPS + pp] = val; });
  __syncthreads();
  // y_p = sum_q Lambda_pq J_q with the reflection signs of the odd components
  const int nh = two ? 2 : 1;
  const T* lt = lam + ((size_t)kyc * kxn + kx0) * KZC * 6;
  for (int idx = threadIdx.x; idx < nh * W * M; idx += blockDim.x) {
    const int hh = idx / (W * M), rem = idx - hh * (W * M);
    const int cc = rem / M, kz = rem - cc * M;
    if (kx0 + cc >= kxn) continue;
    const int kzc = kz <= M / 2 ? kz : M - kz;
    const T sz = kz <= M / 2 ? (T)1 : (T)-1;
    const T sy = hh ? (T)-1 : (T)1;
    const T* Lp = lt + ((size_t)cc * KZC + kzc) * 6;
    const T lxx = Lp[0], lyy = Lp[1], lzz = Lp[2];
    const T lxy = sy * Lp[3], lxz = sz * Lp[4], lyz = sy * sz * Lp[5];
    cpx<T>* q = lds + kz * NPS + hh * 3 * W + cc;
    const cpx<T> jx = q[0], jy = q[W], jz = q[2 * W];
    q[0] = cpx<T>{lxx * jx.x + lxy * jy.x + lxz * jz.x, lxx * jx.y + lxy * jy.y + lxz * jz.y};
    q[W] = cpx<T>{lxy * jx.x + lyy * jy.x + lyz * jz.x, lxy * jx.y + lyy * jy.y + lyz * jz.y};
    q[2 * W] = cpx<T>{lxz * jx.x + lyz * jy.x + lzz * jz.x, lxz * jx.y + lyz * jy.y + lzz * jz.y};
  }
  __syncthreads();
  load_first<T, M>(v, p, jt, [&](int pp, int e) { return lds[e * NPS + pp]; });
  __syncthreads();
  run_fft<T, M, true>(v, lds, tw, p, jt, NPS, [&](int, int e, cpx<T> val) {
    if (ok && e < n_out) dst[(size_t)e * plane] = val;
  });
}

// ------------------------------------------------------------------ dispatch
bool length_supported(int M) {
  switch (M) {
#define X(m) case m:
    MOT_FOR_EACH_LEN(X)
#undef X
    return true;
    default:
      return false;
  }
}

template <typename T, typename IO>
hipError_t x_forward(const IO* in, void* out, int M, int nrows, int rows_per_comp, int ncomp, int row_len,
                     int n_in, int kxs, const void* tw, const void* tw2, hipStream_t s) {
  switch (M) {
#define X(m)                                                                                            \
  case m: {                                                                                             \
    using C = XCfg<T, m>;                                                                               \
    const int nb = (ncomp == 3 && C::NP >= 3) ? (rows_per_comp + C::NP / 3 - 1) / (C::NP / 3)          \
                                              : (nrows + C::NP - 1) / C::NP;                           \
    hipLaunchKernelGGL((k_x_forward<T, IO, m>), dim3(nb), dim3(C::BLOCK), C::LDS, s, in, (cpx<T>*)out, nrows, \
                       rows_per_comp, ncomp, row_len, n_in, kxs, (const cpx<T>*)tw, (const cpx<T>*)tw2);  \
    return hipGetLastError();                                                                           \
  }
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, typename IO>
hipError_t x_inverse(const void* in, IO* y, const IO* J, const double* eps, Epilogue ep, int M, int nrows,
                     int rows_per_comp, int ncomp, int row_len, int n_out, int kxs, const void* tw,
                     const void* tw2, hipStream_t s) {
  switch (M) {
#define X(m)                                                                                            \
  case m: {                                                                                             \
    using C = XCfg<T, m>;                                                                               \
    const int nb = (ncomp == 3 && C::NP >= 3) ? (rows_per_comp + C::NP / 3 - 1) / (C::NP / 3)          \
                                              : (nrows + C::NP - 1) / C::NP;                           \
    hipLaunchKernelGGL((k_x_inverse<T, IO, m>), dim3(nb), dim3(C::BLOCK), C::LDS, s, (const cpx<T>*)in, y, J, \
                       eps, ep, nrows, rows_per_comp, ncomp, row_len, n_out, kxs, (const cpx<T>*)tw,      \
                       (const cpx<T>*)tw2);                                                            \
    return hipGetLastError();                                                                           \
  }
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t y_pass(const void* in, void* out, int M, bool inverse, int kx, int kxs, int planes,
                  int rows_in, int n_in, int rows_out, int n_out, const void* tw, hipStream_t s) {
  switch (M) {
#define X(m)                                                                                         \
  case m: {                                                                                          \
    using C = YCfg<T, m>;                                                                            \
    const int ntx = (kx + C::NP - 1) / C::NP, nlog = ntx * planes;                                   \
    dim3 g(xcd_grid(nlog));                                                                          \
    if (inverse)                                                                                     \
      hipLaunchKernelGGL((k_y_pass<T, m, true>), g, dim3(C::BLOCK), C::LDS, s, (const cpx<T>*)in,     \
                         (cpx<T>*)out, kx, kxs, rows_in, n_in, rows_out, n_out, (const cpx<T>*)tw, ntx,  \
                         nlog);                                                                      \
    else                                                                                             \
      hipLaunchKernelGGL((k_y_pass<T, m, false>), g, dim3(C::BLOCK), C::LDS, s, (const cpx<T>*)in,    \
                         (cpx<T>*)out, kx, kxs, rows_in, n_in, rows_out, n_out, (const cpx<T>*)tw, ntx,  \
                         nlog);                                                                      \
    return hipGetLastError();                                                                        \
  }
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, int M, int NC>
static hipError_t z_launch(const void* in, void* out, int mode, int kx, int kxs, int ny, int rows_in,
                           int n_in, int rows_out, int n_out, const T* lam, const void* tw, hipStream_t s) {
  const cpx<T>* i_ = (const cpx<T>*)in;
  cpx<T>* o_ = (cpx<T>*)out;
  const cpx<T>* t_ = (const cpx<T>*)tw;
  if (mode == Z_FUSED) {
    if (NC != 3) return hipErrorInvalidValue;
    using C = ZFCfg<T, M>;
    const int ntx = (kx + C::W - 1) / C::W, nlog = ntx * (ny / 2 + 1);
    hipLaunchKernelGGL((k_z_fused<T, M>), dim3(xcd_grid(nlog)), dim3(C::BLOCK), C::LDS, s, i_, o_, kx, kxs, ny,
                       rows_in, n_in, rows_out, n_out, lam, t_, ntx, nlog);
    return hipGetLastError();
  }
  using C = ZCfg<T, M, NC>;
  const int ntx = (kx + C::W - 1) / C::W, nlog = ntx * ny;
  dim3 g(xcd_grid(nlog));
  if (mode == Z_FWD)
    hipLaunchKernelGGL((k_z_pass<T, M, NC, false>), g, dim3(C::BLOCK), C::LDS, s, i_, o_, kx, kxs, ny, rows_in,
                       n_in, rows_out, n_out, t_, ntx, nlog);
  else
    hipLaunchKernelGGL((k_z_pass<T, M, NC, true>), g, dim3(C::BLOCK), C::LDS, s, i_, o_, kx, kxs, ny, rows_in,
                       n_in, rows_out, n_out, t_, ntx, nlog);
  return hipGetLastError();
}

template <typename T>
hipError_t z_pass(const void* in, void* out, int M, int mode, int nc, int kx, int kxs, int ny,
                  int rows_in, int n_in, int rows_out, int n_out, const T* lam, const void* tw,
                  hipStream_t s) {
  switch (M) {
#define X(m)                                                                                      \
  case m:                                                                                         \
    return nc == 3 ? z_launch<T, m, 3>(in, out, mode, kx, kxs, ny, rows_in, n_in, rows_out, n_out, \
                                       lam, tw, s)                                                \
                   : z_launch<T, m, 1>(in, out, mode, kx, kxs, ny, rows_in, n_in, rows_out, n_out, \
                                       lam, tw, s);
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

#define XINST(T, IO)                                                                                      \
  template hipError_t x_forward<T, IO>(const IO*, void*, int, int, int, int, int, int, int, const void*,    \
                                       const void*, hipStream_t);                                          \
  template hipError_t x_inverse<T, IO>(const void*, IO*, const IO*, const double*, Epilogue, int, int, int, \
                                       int, int, int, int, const void*, const void*, hipStream_t);
XINST(float, float)
XINST(float, double)
XINST(double, double)
#undef XINST
template hipError_t y_pass<float>(const void*, void*, int, bool, int, int, int, int, int, int, int,
                                  const void*, hipStream_t);
template hipError_t y_pass<double>(const void*, void*, int, bool, int, int, int, int, int, int, int,
                                   const void*, hipStream_t);
template hipError_t z_pass<float>(const void*, void*, int, int, int, int, int, int, int, int, int, int,
                                  const float*, const void*, hipStream_t);
template hipError_t z_pass<double>(const void*, void*, int, int, int, int, int, int, int, int, int, int,
                                   const double*, const void*, hipStream_t);

}  // namespace motfft
