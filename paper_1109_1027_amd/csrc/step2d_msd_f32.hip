// The 2D whole-step kernels for FP32, MSD.
#include "step2d_impl.h"

namespace nlse {

hipError_t launch_step2d_msd_f32(const Step2DArgs &a, hipStream_t st) { return launch_v<float, float, 0, true>(a, st); }

}  // namespace nlse
