// Pass kernels for double, radix family E = 36.
#include "pass_kernels.h"

PSPFFT_FAMILY(double, 36, launch_f64_e36)
