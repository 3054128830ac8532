// nlse_mass_noalloc: the FP64 mass reduction of nlse_mass for a caller's dense device
// field, through a file-scope device array instead of memory the library allocates, for
// callers that cannot allocate (code under HIP graph capture, serving loops that forbid
// hipMalloc).
//
// Scratch.  `scratch` holds the reduction's per-block partial sums (reduce_partials()
// doubles, every one rewritten by the first pass of each call, so nothing has to start at
// zero).  Its size does not depend on the field.  Each GPU holds its own copy for the life
// of the process; its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and only that address is handed to
// kernels.  Calls that overlap on one GPU (two streams, two threads) share the array and
// race; callers serialise them.
#include <cmath>
#include <mutex>

#include "ctx.h"

namespace nlse {
namespace {

constexpr int SCRATCH_DOUBLES = 1024;   // partial sums of the first reduction pass
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (taken on first use).
int scratch_for_current_device(double **out)
{
    int dev = -1;
    HIPTRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(NLSE_E_UNSUPPORTED, "nlse_mass_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hipfail(e, "nlse_mass_noalloc: hipGetSymbolAddress(scratch)");
        if (!p) return fail(NLSE_E_HIP, "nlse_mass_noalloc: scratch has no device address");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return NLSE_OK;
}

}  // namespace
}  // namespace nlse

using namespace nlse;

extern "C" int nlse_mass_noalloc(int32_t ndim, const int64_t *n, double h, int32_t prec, const void *psi,
                                 double *out, void *stream)
{
    if (!n || !psi || !out) return fail(NLSE_E_INVAL, "nlse_mass_noalloc: NULL argument");
    if (ndim < 1 || ndim > 3) return fail(NLSE_E_INVAL, "nlse_mass_noalloc: ndim must be 1, 2 or 3");
    if (!(h > 0.0) || !std::isfinite(h)) return fail(NLSE_E_INVAL, "nlse_mass_noalloc: h must be finite and > 0");
    if (prec != NLSE_F64 && prec != NLSE_F32 && prec != NLSE_F32_MIXED)
        return fail(NLSE_E_INVAL, "nlse_mass_noalloc: unknown precision");
    for (int a = 0; a < ndim; ++a)
        if (n[a] < 1 || n[a] > (int64_t(1) << 40)) return fail(NLSE_E_INVAL, "nlse_mass_noalloc: bad interval count");
    if (reduce_partials() > SCRATCH_DOUBLES)
        return fail(NLSE_E_UNSUPPORTED, "nlse_mass_noalloc: reduction needs more partials than the scratch holds");
    // dense [z][y][x] layout: no row padding, node x = 0 first
    Layout L;
    L.dim = ndim;
    L.nx = n[0];
    L.ny = ndim > 1 ? n[1] : 0;
    L.nz = ndim > 2 ? n[2] : 0;
    L.ox = 0;
    L.px = L.nx + 1;
    L.py = L.ny + 1;
    L.total = L.px * L.py * (L.nz + 1);
    double *partials = nullptr;
    int rc = scratch_for_current_device(&partials);
    if (rc) return rc;
    const Prec pr = prec == NLSE_F32 ? P_F32 : prec == NLSE_F32_MIXED ? P_MIXED : P_F64;
    HIPTRY(launch_mass(pr, psi, L, partials, out, (hipStream_t)stream, std::pow(h, ndim)));
    return NLSE_OK;
}
