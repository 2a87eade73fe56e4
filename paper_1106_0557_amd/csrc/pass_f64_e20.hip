// Pass kernels for double, radix family E = 20.
#include "plane_kernels.h"

PSPFFT_FAMILY(double, 20, launch_f64_e20, plane_f64_e20)
