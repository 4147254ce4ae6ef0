// x pass of the circulant-embedded Green product: entry points.  Tile
// variant 0 is instantiated here, variant 1 in fft_x_alt.hip, and the forms
// with fused solver work in fft_x_solver.hip (variant 0) and
// fft_x_solver_alt.hip (variant 1).
#include "fft_x_kernels.h"

namespace motfft {

MOT_X_VARIANT(0)

#define MOT_X_EXT_FWD(T, IO, V, KM)                                                                          \
  extern template hipError_t x_forward_v<T, IO, V, KM>(const IO*, void*, int, int, int, int, int, int, int,   \
                                                       const void*, const void*, hipStream_t, const double*,  \
                                                       Gate, const Krylov&);
#define MOT_X_EXT_INV(T, IO, V, KM)                                                                          \
  extern template hipError_t x_inverse_v<T, IO, V, KM>(const void*, IO*, const IO*, const T*, Epilogue,  \
                                                       int, int, int, int, int, int, int, const void*,        \
                                                       const void*, hipStream_t, Gate, const Krylov&);
MOT_X_EXT_FWD(float, float, 1, KRY_NONE)
MOT_X_EXT_FWD(float, double, 1, KRY_NONE)
MOT_X_EXT_FWD(double, double, 1, KRY_NONE)
MOT_X_EXT_INV(float, float, 1, KRY_NONE)
MOT_X_EXT_INV(float, double, 1, KRY_NONE)
MOT_X_EXT_INV(double, double, 1, KRY_NONE)
#define MOT_X_EXT_SOLVER(T, V)       \
  MOT_X_EXT_FWD(T, T, V, KRY_HALF0)  \
  MOT_X_EXT_FWD(T, T, V, KRY_U)      \
  MOT_X_EXT_FWD(T, T, V, KRY_XFIX)   \
  MOT_X_EXT_FWD(T, T, V, KRY_SCALE)  \
  MOT_X_EXT_INV(T, T, V, KRY_HALF1)  \
  MOT_X_EXT_INV(T, T, V, KRY_V)      \
  MOT_X_EXT_INV(T, T, V, KRY_SCALE)
MOT_X_EXT_SOLVER(float, 0)
MOT_X_EXT_SOLVER(double, 0)
MOT_X_EXT_SOLVER(float, 1)
MOT_X_EXT_SOLVER(double, 1)
MOT_X_EXT_INV(double, double, 0, KRY_RESID)
MOT_X_EXT_INV(double, double, 1, KRY_RESID)

namespace {
const Krylov kNoSolver{};

template <typename T, typename IO, int V>
hipError_t x_forward_k(const IO* in, void* out, int M, int nrows, int rows_per_comp, int ncomp, int row_len,
                       int n_in, int kxs, const void* tw, const void* tw2, hipStream_t s, const double* pre,
                       Gate gg, const Krylov* kry) {
  const int mode = kry ? kry->mode : KRY_NONE;
  if (mode == KRY_NONE)
    return x_forward_v<T, IO, V, KRY_NONE>(in, out, M, nrows, rows_per_comp, ncomp, row_len, n_in, kxs, tw, tw2,
                                           s, pre, gg, kNoSolver);
  if constexpr (std::is_same<T, IO>::value) {
#define F(KM)                                                                                                 \
  if (mode == KM)                                                                                             \
    return x_forward_v<T, IO, V, KM>(in, out, M, nrows, rows_per_comp, ncomp, row_len, n_in, kxs, tw, tw2, s, \
                                     pre, gg, *kry);
    F(KRY_HALF0)
    F(KRY_U)
    F(KRY_XFIX)
    F(KRY_SCALE)
#undef F
  }
  return hipErrorInvalidValue;
}

template <typename T, typename IO, int V>
hipError_t x_inverse_k(const void* in, IO* y, const IO* J, const T* eps, Epilogue ep, int M, int nrows,
                       int rows_per_comp, int ncomp, int row_len, int n_out, int kxs, const void* tw,
                       const void* tw2, hipStream_t s, Gate gg, const Krylov* kry) {
  const int mode = kry ? kry->mode : KRY_NONE;
  if (mode == KRY_NONE)
    return x_inverse_v<T, IO, V, KRY_NONE>(in, y, J, eps, ep, M, nrows, rows_per_comp, ncomp, row_len, n_out, kxs,
                                           tw, tw2, s, gg, kNoSolver);
  if constexpr (std::is_same<T, IO>::value) {
#define F(KM)                                                                                                  \
  if (mode == KM)                                                                                              \
    return x_inverse_v<T, IO, V, KM>(in, y, J, eps, ep, M, nrows, rows_per_comp, ncomp, row_len, n_out, kxs, tw, \
                                     tw2, s, gg, *kry);
    F(KRY_HALF1)
    F(KRY_V)
    F(KRY_SCALE)
    if constexpr (sizeof(T) == 8) F(KRY_RESID)
#undef F
  }
  return hipErrorInvalidValue;
}
}  // namespace

template <typename T, typename IO>
hipError_t x_forward(const IO* in, void* out, int M, int nrows, int rows_per_comp, int ncomp, int row_len,
                     int n_in, int kxs, const void* tw, const void* tw2, hipStream_t s, const double* pre,
                     Gate gg, int var, const Krylov* kry) {
  if (var == 1 && 2 * n_in == M)
    return x_forward_k<T, IO, 1>(in, out, M, nrows, rows_per_comp, ncomp, row_len, n_in, kxs, tw, tw2, s, pre, gg,
                                 kry);
  if (var != 0 && var != 1) return hipErrorInvalidValue;
  return x_forward_k<T, IO, 0>(in, out, M, nrows, rows_per_comp, ncomp, row_len, n_in, kxs, tw, tw2, s, pre, gg,
                               kry);
}

template <typename T, typename IO>
hipError_t x_inverse(const void* in, IO* y, const IO* J, const T* eps, Epilogue ep, int M, int nrows,
                     int rows_per_comp, int ncomp, int row_len, int n_out, int kxs, const void* tw,
                     const void* tw2, hipStream_t s, Gate gg, int var, const Krylov* kry) {
  if (var == 1)
    return x_inverse_k<T, IO, 1>(in, y, J, eps, ep, M, nrows, rows_per_comp, ncomp, row_len, n_out, kxs, tw, tw2,
                                 s, gg, kry);
  if (var != 0) return hipErrorInvalidValue;
  return x_inverse_k<T, IO, 0>(in, y, J, eps, ep, M, nrows, rows_per_comp, ncomp, row_len, n_out, kxs, tw, tw2, s,
                               gg, kry);
}

int x_pass_blocks(int M, bool f64, int var, int nrows, int rows_per_comp, int ncomp) {
  if (var == 1) return x_pass_blocks_v<1>(M, f64, nrows, rows_per_comp, ncomp);
  if (var != 0) return 0;
  return x_pass_blocks_v<0>(M, f64, nrows, rows_per_comp, ncomp);
}

#define XINST(T, IO)                                                                                      \
  template hipError_t x_forward<T, IO>(const IO*, void*, int, int, int, int, int, int, int, const void*,    \
                                       const void*, hipStream_t, const double*, Gate, int, const Krylov*); \
  template hipError_t x_inverse<T, IO>(const void*, IO*, const IO*, const T*, Epilogue, int, int, int, \
                                       int, int, int, int, const void*, const void*, hipStream_t, Gate, int, \
                                       const Krylov*);
XINST(float, float)
XINST(float, double)
XINST(double, double)
#undef XINST

}  // namespace motfft
