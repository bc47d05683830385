// Sweep kernels of 3D problems in double arithmetic (one translation unit per
// dimension and precision, so the library's kernels compile in parallel).
#include "gpweno_sweep.h"

namespace gpw {

hipError_t launch_sweep_3d_f64(const LaunchSel& k, const void* args, long long blocks, hipStream_t s) {
    return launch_r<3, double>(k, args, blocks, s);
}

}  // namespace gpw
