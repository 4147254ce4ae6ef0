// x pass, tile variant 1 (see XCfg).
#include "fft_x_kernels.h"

namespace motfft {
MOT_X_VARIANT(1)
}  // namespace motfft
