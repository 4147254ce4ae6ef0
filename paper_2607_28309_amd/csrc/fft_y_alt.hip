// y pass, tile variant 1 (see YCfg).
#include "fft_y_kernels.h"

namespace motfft {
MOT_Y_VARIANT(1)
}  // namespace motfft
