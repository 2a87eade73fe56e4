// Pass kernels for float, radix family E = 16.
#include "pass_kernels.h"

PSPFFT_FAMILY(float, 16, launch_f32_e16)
