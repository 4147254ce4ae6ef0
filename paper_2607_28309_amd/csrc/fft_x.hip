// x pass of the circulant-embedded Green product: entry points (tile
// variant 0 is instantiated here, variant 1 in fft_x_alt.hip).
#include "fft_x_kernels.h"

namespace motfft {

MOT_X_VARIANT(0)

#define MOT_X_EXTERN(T, IO)                                                                                     \
  extern template hipError_t x_forward_v<T, IO, 1>(const IO*, void*, int, int, int, int, int, int, int,         \
                                                   const void*, const void*, hipStream_t, const double*, Gate); \
  extern template hipError_t x_inverse_v<T, IO, 1>(const void*, IO*, const IO*, const double*, Epilogue, int,   \
                                                   int, int, int, int, int, int, const void*, const void*,      \
                                                   hipStream_t, Gate);
MOT_X_EXTERN(float, float)
MOT_X_EXTERN(float, double)
MOT_X_EXTERN(double, double)
#undef MOT_X_EXTERN

template <typename T, typename IO>
hipError_t x_forward(const IO* in, void* out, int M, int nrows, int rows_per_comp, int ncomp, int row_len,
                     int n_in, int kxs, const void* tw, const void* tw2, hipStream_t s, const double* pre,
                     Gate gg, int var) {
  if (var == 1 && 2 * n_in == M)
    return x_forward_v<T, IO, 1>(in, out, M, nrows, rows_per_comp, ncomp, row_len, n_in, kxs, tw, tw2, s, pre, gg);
  if (var != 0 && var != 1) return hipErrorInvalidValue;
  return x_forward_v<T, IO, 0>(in, out, M, nrows, rows_per_comp, ncomp, row_len, n_in, kxs, tw, tw2, s, pre, gg);
}

template <typename T, typename IO>
hipError_t x_inverse(const void* in, IO* y, const IO* J, const double* eps, Epilogue ep, int M, int nrows,
                     int rows_per_comp, int ncomp, int row_len, int n_out, int kxs, const void* tw,
                     const void* tw2, hipStream_t s, Gate gg, int var) {
  if (var == 1)
    return x_inverse_v<T, IO, 1>(in, y, J, eps, ep, M, nrows, rows_per_comp, ncomp, row_len, n_out, kxs, tw, tw2,
                                 s, gg);
  if (var != 0) return hipErrorInvalidValue;
  return x_inverse_v<T, IO, 0>(in, y, J, eps, ep, M, nrows, rows_per_comp, ncomp, row_len, n_out, kxs, tw, tw2, s,
                               gg);
}

#define XINST(T, IO)                                                                                      \
  template hipError_t x_forward<T, IO>(const IO*, void*, int, int, int, int, int, int, int, const void*,    \
                                       const void*, hipStream_t, const double*, Gate, int);                \
  template hipError_t x_inverse<T, IO>(const void*, IO*, const IO*, const double*, Epilogue, int, int, int, \
                                       int, int, int, int, const void*, const void*, hipStream_t, Gate, int);
XINST(float, float)
XINST(float, double)
XINST(double, double)
#undef XINST

}  // namespace motfft
