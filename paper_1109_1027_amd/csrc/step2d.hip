// Entry of the 2D whole-step kernel (one launch per RK4 step; the scheme is described in
// step2d_impl.h): dispatch to the translation unit that instantiates the kernels of the context's
// precision and boundary rule.
#include "kernels.h"

namespace nlse {

int step2d_variants() { return 7; }

hipError_t launch_step2d(Prec prec, const Step2DArgs &a, hipStream_t st)
{
    if (a.msd) {
        if (a.stencil != 0) return hipErrorInvalidValue;   // MSD with the per-axis 2SHOC form
        switch (prec) {
        case P_F64: return launch_step2d_msd_f64(a, st);
        case P_F32: return launch_step2d_msd_f32(a, st);
        default: return launch_step2d_msd_mixed(a, st);
        }
    }
    switch (prec) {
    case P_F64: return launch_step2d_f64(a, st);
    case P_F32: return launch_step2d_f32(a, st);
    default: return launch_step2d_mixed(a, st);
    }
}

}  // namespace nlse
