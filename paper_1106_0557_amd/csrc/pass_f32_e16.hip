// Pass kernels for float, radix family E = 16.
#include "plane_kernels.h"

PSPFFT_FAMILY(float, 16, launch_f32_e16, plane_f32_e16)
