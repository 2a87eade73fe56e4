// Pass kernels for double, radix family E = 36.
#include "plane_kernels.h"

PSPFFT_FAMILY(double, 36, launch_f64_e36, plane_f64_e36)
