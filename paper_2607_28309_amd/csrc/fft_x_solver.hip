// x pass, forms with fused solver work (see Krylov), tile variant 0.
#include "fft_x_kernels.h"

namespace motfft {
MOT_X_SOLVER_T(float, 0)
MOT_X_SOLVER_T(double, 0)
MOT_X_RESID(0)
}  // namespace motfft
