// The 2D whole-step kernels for mixed precision, Dirichlet (every Laplacian).
#include "step2d_impl.h"

namespace nlse {

hipError_t launch_step2d_mixed(const Step2DArgs &a, hipStream_t st) { return launch_dirichlet<float, double>(a, st); }

}  // namespace nlse
