// Sweep kernels of 2D problems in float arithmetic (one translation unit per
// dimension and precision, so the library's kernels compile in parallel).
#include "gpweno_sweep.h"

namespace gpw {

hipError_t launch_sweep_2d_f32(const LaunchSel& k, const void* args, long long blocks, hipStream_t s) {
    return launch_r<2, float>(k, args, blocks, s);
}

}  // namespace gpw
