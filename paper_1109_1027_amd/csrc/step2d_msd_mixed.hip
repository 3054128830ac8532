// The 2D whole-step kernels for mixed precision, MSD.
#include "step2d_impl.h"

namespace nlse {

hipError_t launch_step2d_msd_mixed(const Step2DArgs &a, hipStream_t st) { return launch_v<float, double, 0, true>(a, st); }

}  // namespace nlse
