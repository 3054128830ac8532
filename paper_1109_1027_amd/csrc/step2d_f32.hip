// The 2D whole-step kernels for FP32, Dirichlet (every Laplacian).
#include "step2d_impl.h"

namespace nlse {

hipError_t launch_step2d_f32(const Step2DArgs &a, hipStream_t st) { return launch_dirichlet<float, float>(a, st); }

}  // namespace nlse
