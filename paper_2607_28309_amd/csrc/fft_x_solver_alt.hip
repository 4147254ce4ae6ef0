// x pass, forms with fused solver work (see Krylov), tile variant 1.
#include "fft_x_kernels.h"

namespace motfft {
MOT_X_SOLVER_T(float, 1)
MOT_X_SOLVER_T(double, 1)
MOT_X_RESID(1)
}  // namespace motfft
