// Pass kernels for double, radix family E = 16.
#include "plane_kernels.h"

PSPFFT_FAMILY(double, 16, launch_f64_e16, plane_f64_e16)
