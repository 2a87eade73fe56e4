// Pass kernels for float, radix family E = 20.
#include "pass_kernels.h"

PSPFFT_FAMILY(float, 20, launch_f32_e20)
