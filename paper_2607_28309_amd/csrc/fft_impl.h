// Shared configuration of the FFT pass kernels (x, y and z passes live in
// their own translation units so that they compile in parallel).
//
// Workgroups of the y and z passes are issued in an XCD-aware order: the
// hardware hands consecutive workgroup ids to the eight XCDs in turn, each
// with its own L2, so logical tile t is given to id (t mod Q) * 8 + t / Q
// (Q = ceil(tiles/8)); neighbouring kx tiles of one row then share an L2 and
// the 128-byte lines they split are fetched from HBM once.
#pragma once

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
//
// Tile-shape variants (chosen per context by the autotuner): V = 0 is the
// default shape.  V = 1: the x pass takes 3 (NP0 / 4) rows (whole voxel rows
// of all three components, fewer rows per workgroup); the y pass exchanges
// real and imaginary parts in turn through a buffer of half the bytes and
// doubles its columns when the doubled tile fits a workgroup (twice the
// pencils in flight per CU); the z passes without the spectral multiply do
// the same split with their variant-0 tile; the fused z pass halves its
// columns (twice the workgroups, half the LDS each).
constexpr size_t LDS_MAX = 160 * 1024;
template <typename T, int M, int V = 0> struct XCfg {
  static constexpr int TJ = PlanInfo<M>::TJ;
  static constexpr int SZ = (int)sizeof(cpx<T>);
  static constexpr int NP0 =
      cmax(1, floor_pow2(cmin(256 / TJ, (LDS_BUDGET - (2 * M + 1) * SZ) / ((M + 1) * SZ) - 1)));
  static constexpr int NP = V == 0 ? NP0 : (NP0 >= 4 ? 3 * (NP0 / 4) : cmax(1, NP0 / 2));
  static constexpr int NPS = NP + 1;
  static constexpr int BLOCK = NP * TJ;
  // swizzled exchange slots (lslot) for FP32 when the row count allows them
  // (FP32 products 0.368 -> 0.362 ms at 320x320x48; FP64 unchanged)
  static constexpr int SW = sizeof(T) == 4 && NP % 4 == 0 ? 1 : 0;
  // FP64: the twiddle tables are read from global memory (L1/L2) instead
  // of LDS, which leaves room for more rows per CU
  static constexpr bool TWG = sizeof(T) == 8;
  static constexpr size_t LDS = (size_t)((M + 1) * NPS + (TWG ? 0 : 2 * M + 1)) * SZ;
};
template <typename T, int M, int V = 0> struct YCfg {
  static constexpr int TJ = PlanInfo<M>::TJ;
  static constexpr int SZ = (int)sizeof(cpx<T>);
  static constexpr int NP0 = cmax(1, floor_pow2(cmin(cmin(256 / TJ, 32), (LDS_BUDGET - M * SZ) / (M * SZ) - 1)));
  // variant 1: split exchanges (real parts, then imaginary parts) and twice
  // the columns when that fits a workgroup
  static constexpr bool SPLIT = V == 1;
  static constexpr int NP = V == 0 ? NP0 : (2 * NP0 * TJ <= 1024 ? 2 * NP0 : NP0);
  static constexpr int NPS = NP + 1;
  static constexpr int BLOCK = NP * TJ;
  static constexpr size_t BUF = (size_t)M * NPS * (SPLIT ? sizeof(T) : sizeof(cpx<T>));  // exchange buffer bytes
  // FP64: the twiddle table is read from global memory (as in XCfg)
  static constexpr bool TWG = sizeof(T) == 8;
  static constexpr size_t LDS = BUF + (TWG ? 0 : (size_t)M * SZ);
  static_assert(BUF % sizeof(cpx<T>) == 0, "the twiddle table after the buffer is aligned");
};
template <typename T, int M, int NC, int V = 0> struct ZCfg {
  static constexpr int TJ = PlanInfo<M>::TJ;
  static constexpr int SZ = (int)sizeof(cpx<T>);
  static constexpr int W0 =
      cmax(1, floor_pow2(cmin(cmin(16, 1024 / (NC * TJ)), (LDS_BUDGET - 2 * M * SZ) / (NC * M * SZ))));
  // variant 1: the same tile with split exchanges (half the LDS bytes)
  static constexpr bool SPLIT = V == 1;
  static constexpr int W = W0;
  static constexpr int NP = NC * W;
  static constexpr int NPS = NP + 1;
  static constexpr int BLOCK = NP * TJ;
  static constexpr size_t BUF = (size_t)M * NPS * (SPLIT ? sizeof(T) : sizeof(cpx<T>));  // exchange buffer bytes
  static constexpr size_t LDS = BUF + (size_t)M * SZ;
  static_assert(BUF % sizeof(cpx<T>) == 0, "the twiddle table after the buffer is aligned");
};

// z pass with the spectral multiply: W kx columns x 3 components x 2 ky rows.
template <typename T, int M, int V = 0> struct ZFCfg {
  static constexpr int TJ = PlanInfo<M>::TJ;
  static constexpr int SZ = (int)sizeof(cpx<T>);
  static constexpr int W0 =
      cmax(1, floor_pow2(cmin(cmin(16, 1024 / (6 * TJ)), (LDS_BUDGET - 2 * M * SZ) / (6 * M * SZ))));
  static constexpr int W = V == 0 ? W0 : cmax(1, W0 / 2);
  static constexpr int NP = 6 * W;
  static constexpr int NPS = NP + 1;
  static constexpr int BLOCK = NP * TJ;
  static constexpr size_t LDS = (size_t)(M * NPS + M) * SZ;
};

// The buffer between the y and z passes: element (plane pl, row r, column
// kx) of P planes (component-major, pl = comp * rows + z) sits at
//   ((r * NT + kx / 16) * P + pl) * 16 + kx % 16,   NT = kxs / 16,
// so that a z pass reads and writes each (ky, 16-column block) as one
// contiguous range of P * 16 values (a z pencil has stride 16); the y passes
// step from row to row by NT * P * 16.  (kxs is a multiple of 16.)
__host__ __device__ inline size_t yz_index(int pl, int r, int kx, int kxs, int P) {
  return (((size_t)r * (kxs >> 4) + (kx >> 4)) * P + pl) * 16 + (kx & 15);
}
__host__ __device__ inline size_t yz_row_stride(int kxs, int P) { return (size_t)(kxs >> 4) * P * 16; }

constexpr int NXCD = 8;
// logical tile of workgroup id b; tiles >= nlog are idle
__device__ __forceinline__ int xcd_tile(int b, int nlog) {
  const int q = (nlog + NXCD - 1) / NXCD;
  return (b % NXCD) * q + b / NXCD;
}
inline int xcd_grid(int nlog) { return ((nlog + NXCD - 1) / NXCD) * NXCD; }

// Copy a table of N entries into LDS: all loads of a thread are issued
// before its LDS writes.
template <typename C, int N, int BLOCK>
__device__ __forceinline__ void load_table(C* dst, const C* __restrict__ src) {
  constexpr int IT = (N + BLOCK - 1) / BLOCK;
  C tmp[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int idx = (int)threadIdx.x + i * BLOCK;
    tmp[i] = src[idx < N ? idx : N - 1];
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int idx = (int)threadIdx.x + i * BLOCK;
    if (idx < N) dst[idx] = tmp[i];
  }
}

template <typename IO> struct io2;
template <> struct io2<float> { using t = float2; };
template <> struct io2<double> { using t = double2; };

}  // namespace motfft
