// Pass kernels for float, radix family E = 24.
#include "plane_kernels.h"

PSPFFT_FAMILY(float, 24, launch_f32_e24, plane_f32_e24)
