// y pass of the circulant-embedded Green product: entry points (tile
// variant 0 is instantiated here, variant 1 in fft_y_alt.hip).
#include "fft_y_kernels.h"

namespace motfft {

MOT_Y_VARIANT(0)

extern template hipError_t y_pass_v<float, 1>(const void*, void*, int, bool, int, int, int, int, int, int, int,
                                              const void*, hipStream_t, Gate);
extern template hipError_t y_pass_v<double, 1>(const void*, void*, int, bool, int, int, int, int, int, int, int,
                                               const void*, hipStream_t, Gate);

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

template <typename T>
hipError_t y_pass(const void* in, void* out, int M, bool inverse, int kx, int kxs, int planes,
                  int rows_in, int n_in, int rows_out, int n_out, const void* tw, hipStream_t s, Gate g, int var) {
  const bool full_fwd = !inverse && n_in == M;
  if (var == 1 && !full_fwd)
    return y_pass_v<T, 1>(in, out, M, inverse, kx, kxs, planes, rows_in, n_in, rows_out, n_out, tw, s, g);
  if (var != 0 && var != 1) return hipErrorInvalidValue;
  return y_pass_v<T, 0>(in, out, M, inverse, kx, kxs, planes, rows_in, n_in, rows_out, n_out, tw, s, g);
}

template hipError_t y_pass<float>(const void*, void*, int, bool, int, int, int, int, int, int, int,
                                  const void*, hipStream_t, Gate, int);
template hipError_t y_pass<double>(const void*, void*, int, bool, int, int, int, int, int, int, int,
                                   const void*, hipStream_t, Gate, int);

}  // namespace motfft
