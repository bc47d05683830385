// Sweep kernels of 3D problems in float arithmetic (one translation unit per
// dimension and precision, so the library's kernels compile in parallel).
#include "gpweno_sweep.h"

namespace gpw {

hipError_t launch_sweep_3d_f32(int dir, int R, bool fin, int ik, bool bcg, const void* args, hipStream_t s) {
    return launch_r<3, float>(dir, R, fin, ik, bcg, args, s);
}

hipError_t launch_sweep_batch_3d_f32(int dir, int R, bool fin, int ik, bool bcg, const void* args,
                                        long long blocks, hipStream_t s) {
    return launch_batch_r<3, float>(dir, R, fin, ik, bcg, args, blocks, s);
}

}  // namespace gpw
