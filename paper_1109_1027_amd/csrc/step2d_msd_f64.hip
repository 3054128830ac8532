// The 2D whole-step kernels for FP64, MSD.
#include "step2d_impl.h"

namespace nlse {

hipError_t launch_step2d_msd_f64(const Step2DArgs &a, hipStream_t st) { return launch_v<double, double, 0, true>(a, st); }

}  // namespace nlse
