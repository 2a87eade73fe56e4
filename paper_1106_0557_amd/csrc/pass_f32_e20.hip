// Pass kernels for float, radix family E = 20.
#include "plane_kernels.h"

PSPFFT_FAMILY(float, 20, launch_f32_e20, plane_f32_e20)
