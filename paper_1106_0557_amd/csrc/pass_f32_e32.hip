// Pass kernels for float, radix family E = 32: only the z pass of lines of
// 2048 points (radices 32, 32, 2), kept within one wavefront (wave_col_kernel;
// the plan keeps its spectrum kz-fastest).
#include "pass_kernels.h"

namespace pspfft {

hipError_t launch_f32_e32(int mode, int K, int fix, const LaunchArgs &args, int grid, int block, size_t lds,
                          hipStream_t stream) {
    (void)grid;
    (void)block;
    (void)lds;
    if (mode != Z_CONV || !args.wave_z) return hipErrorInvalidValue;
    constexpr int W = kFixWide;
    if (K == 2 && fix == 3) return launch_wave_col<float, 32, 2, Z_CONV, 3>(args, stream);
    if (K == 2 && fix == 3 + W) return launch_wave_col<float, 32, 2, Z_CONV, 3, true>(args, stream);
    return hipErrorInvalidValue;
}

static_assert(wave_col_fits<float, 32, 2, Z_CONV, 3>(), "the 32-family z lines fit the wavefront-owned kernel");

}  // namespace pspfft
