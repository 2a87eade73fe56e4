// Pass kernels for float, radix family E = 36.
#include "pass_kernels.h"

PSPFFT_FAMILY(float, 36, launch_f32_e36)
