// The 2D whole-step kernels for FP64, Dirichlet (every Laplacian).
#include "step2d_impl.h"

namespace nlse {

hipError_t launch_step2d_f64(const Step2DArgs &a, hipStream_t st) { return launch_dirichlet<double, double>(a, st); }

}  // namespace nlse
