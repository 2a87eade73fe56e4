// Pass kernels for double, radix family E = 24.
#include "plane_kernels.h"

PSPFFT_FAMILY(double, 24, launch_f64_e24, plane_f64_e24)
