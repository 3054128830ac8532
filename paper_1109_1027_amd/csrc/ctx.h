// Internal: the context object behind nlse_ctx and the error helpers shared by the
// translation units that implement the C ABI.
#pragma once

#include <string>
#include <vector>

#include "kernels.h"
#include "../../include/nlse.h"

namespace nlse {

int fail(int code, const std::string &msg);
int hipfail(hipError_t e, const char *what);
Coeffs base_coeffs(const nlse_params &p);

}  // namespace nlse

#define HIPTRY(call)                                                \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return nlse::hipfail(e_, #call);      \
    } while (0)

struct nlse_ctx {
    nlse_params p;
    nlse::Layout L;
    nlse::Prec prec;
    size_t esR, esM, rR;        // bytes: stage complex, master complex, stage real
    void *psi = nullptr, *A = nullptr, *B = nullptr, *K = nullptr, *V = nullptr;
    void *psi2 = nullptr;       // second master buffer of the 2D whole-step and 3D pair kernels (swapped with psi)
    void *V0 = nullptr;         // 2D without potential: zeros, read by the whole-step kernel
    void *DB[3] = {nullptr, nullptr, nullptr};
    double *red = nullptr;      // reduction partials (2 * reduce_partials()) + result slots
    hipStream_t stream = nullptr;
    double kmax = 0.0;
    bool have_field = false;
    int variant = 0;            // kernel variant (tile shape; in 2D also stage vs whole-step kernels)
    int stencil = 0;            // 2D Laplacian: NLSE_STENCIL_*
};
