// z pass of the circulant-embedded Green product: entry points (tile
// variant 0 is instantiated here, variant 1 in fft_z_alt.hip).
#include "fft_z_kernels.h"

namespace motfft {

MOT_Z_VARIANT(0)

extern template hipError_t z_pass_v<float, 1>(const void*, void*, int, int, int, int, int, int, int, int, int,
                                              int, const float*, const void*, hipStream_t, Gate);
extern template hipError_t z_pass_v<double, 1>(const void*, void*, int, int, int, int, int, int, int, int, int,
                                               int, const double*, const void*, hipStream_t, Gate);

int z_fused_width(int M, bool f64, int var) {
  if (var != 0 && var != 1) return 0;
  switch (M) {
#define X(m)                                                                      \
  case m:                                                                         \
    if (var == 1) return f64 ? ZFCfg<double, m, 1>::W : ZFCfg<float, m, 1>::W;    \
    return f64 ? ZFCfg<double, m, 0>::W : ZFCfg<float, m, 0>::W;
    MOT_FOR_EACH_LEN(X)
#undef X
    default:
      return 0;
  }
}

template <typename T>
hipError_t z_pass(const void* in, void* out, int M, int mode, int nc, int kx, int kxs, int ny, int rows_in,
                  int n_in, int rows_out, int n_out, const T* lam, const void* tw, hipStream_t s, Gate g, int var) {
  if (var == 1 && nc == 3)
    return z_pass_v<T, 1>(in, out, M, mode, nc, kx, kxs, ny, rows_in, n_in, rows_out, n_out, lam, tw, s, g);
  if (var != 0 && var != 1) return hipErrorInvalidValue;
  return z_pass_v<T, 0>(in, out, M, mode, nc, kx, kxs, ny, rows_in, n_in, rows_out, n_out, lam, tw, s, g);
}

template hipError_t z_pass<float>(const void*, void*, int, int, int, int, int, int, int, int, int, int,
                                  const float*, const void*, hipStream_t, Gate, int);
template hipError_t z_pass<double>(const void*, void*, int, int, int, int, int, int, int, int, int, int,
                                   const double*, const void*, hipStream_t, Gate, int);

}  // namespace motfft
