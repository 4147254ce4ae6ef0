// z passes, tile variant 1 (see ZCfg, ZFCfg).
#include "fft_z_kernels.h"

namespace motfft {
MOT_Z_VARIANT(1)
}  // namespace motfft
