// Pass kernels for float, radix family E = 36.
#include "plane_kernels.h"

PSPFFT_FAMILY(float, 36, launch_f32_e36, plane_f32_e36)
