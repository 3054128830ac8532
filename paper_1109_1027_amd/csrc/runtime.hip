// Host runtime and C ABI of the 2SHOC-RK4 library (declarations in include/nlse.h).
//
// A context owns, in the padded device layout of common.h:
//   psi   master Psi^n            (complex128 for F64 / MIXED, complex64 for F32)
//   A, B  ping-pong stage fields  (complex in the stage precision)
//   K     K_tot                   (stage precision)
//   V     potential               (real, stage precision; absent when V = 0)
//   DB    boundary-face closure values of the per-axis 2SHOC (2D / 3D)
//   psi2  2D, and 3D under Dirichlet: a second master buffer for the 2D whole-step
//         and 3D two-stage kernels
// With the stage-kernel variants one RK4 step enqueues four fused stage kernels:
//   S1 psi -> A, S2 A -> B, S3 B -> A, S4 A -> psi
// (under MSD each preceded by the boundary launch of msd.hip).  The ping-pong keeps
// every stage's stencil input read-only while the next stage field is written.
// The 2D whole-step variants enqueue one kernel per step, psi -> psi2; the 3D
// two-stage variants two, psi -> K, B and B, K, psi -> psi2; both then swap the
// two master pointers.  1D contexts run all steps in one persistent launch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "ctx.h"

using namespace nlse;

namespace {
thread_local std::string g_err;
}  // namespace

namespace nlse {

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hipfail(hipError_t e, const char *what)
{
    return fail(NLSE_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace nlse

Coeffs nlse::base_coeffs(const nlse_params &p)
{
    Coeffs c;
    c.a = p.a;
    c.s = p.s;
    c.ih2 = 1.0 / (p.h * p.h);
    c.c76 = 7.0 / 6.0;
    c.c112 = 1.0 / 12.0;
    c.ia = 1.0 / p.a;
    c.ck = 0.0;
    return c;
}

static int64_t face_nodes(const Layout &L, int axis)
{
    const int64_t nn[3] = {L.nx, L.ny, L.nz};
    int64_t f = 1;
    for (int b = 0; b < L.dim; ++b)
        if (b != axis) f *= nn[b] + 1;
    return f;
}

static void free_ctx(nlse_ctx *c)
{
    if (!c) return;
    void *bufs[] = {c->psi, c->psi2, c->A, c->B, c->K, c->V, c->V0, c->DB[0], c->DB[1], c->DB[2], c->red};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete c;
}

// Autotuner results shared by every context of the same shape in the process.
using TuneKey = std::tuple<int, int, int64_t, int64_t, int64_t, int, int>;   // dim, precision, n, stencil, bc
static std::map<TuneKey, int> g_tuned;
static std::mutex g_tuned_mu;

static TuneKey tune_key(const nlse_ctx *c)
{
    return TuneKey(c->p.ndim, (int)c->prec, c->L.nx, c->L.ny, c->L.nz, c->stencil, (int)c->p.bc);
}

static hipError_t launch_stage(nlse_ctx *c, int stage, double dt, int variant)
{
    const double ck[4] = {dt / 2.0, dt / 2.0, dt, dt / 6.0};
    void *ins[4] = {c->psi, c->A, c->B, c->A};
    void *outs[4] = {c->A, c->B, c->A, nullptr};
    StageArgs a;
    a.in = ins[stage - 1];
    a.out = outs[stage - 1];
    a.psin = c->psi;
    a.K = c->K;
    a.V = c->V;
    for (int d = 0; d < 3; ++d) a.DB[d] = c->DB[d];
    a.L = c->L;
    a.c = base_coeffs(c->p);
    a.c.ck = ck[stage - 1];
    a.stage = stage;
    a.variant = variant;
    a.stencil = c->stencil;
    const bool msd = c->p.bc == NLSE_BC_MSD;
    if (msd) {   // face values of this stage's input (Eq. msdbc_lap) and the boundary nodes (Eq. msdbc_ut)
        hipError_t e = launch_msd_stage(c->prec, a, c->DB, c->stream);
        if (e != hipSuccess) return e;
    }
    return c->p.ndim == 2 ? launch_stage2d(c->prec, a, c->stream) : launch_stage3d(c->prec, a, c->stream);
}

// 2D variants: [0, stage2d_variants()) are the stage kernels, the rest the
// whole-step kernels (their 32-bit offsets need fields below 2^31 elements).
static bool step2d_ok(const nlse_ctx *c)
{
    const bool bc_ok = c->p.bc == NLSE_BC_DIRICHLET || (c->p.bc == NLSE_BC_MSD && c->L.nx >= 2 && c->L.ny >= 2);
    return c->p.ndim == 2 && bc_ok && c->L.total < (int64_t(1) << 31);
}

// 3D variants: [0, stage3d_variants()) the stage kernels, the rest the two-stage pairs
// (2SHOC, Dirichlet, 32-bit offsets).
static bool step3d_ok(const nlse_ctx *c)
{
    return c->p.ndim == 3 && c->stencil == NLSE_STENCIL_2SHOC && c->p.bc == NLSE_BC_DIRICHLET &&
           c->L.total < (int64_t(1) << 31);
}

static int variant_count(const nlse_ctx *c)
{
    if (c->p.ndim == 2) return stage2d_variants() + (step2d_ok(c) ? step2d_variants() : 0);
    if (c->p.ndim == 3) return stage3d_variants() + (step3d_ok(c) ? step3d_variants() : 0);
    return solve1d_variants(c->prec, c->L.nx + 1);
}

// Variants that write Psi^{n+1} into the second master buffer (2D whole step, 3D pairs).
static bool whole_step(const nlse_ctx *c, int variant)
{
    return (c->p.ndim == 2 && variant >= stage2d_variants()) || (c->p.ndim == 3 && variant >= stage3d_variants());
}

// One RK4 step of a 3D context as two launches of two fused stages: psi -> psi2, then swap.
static hipError_t launch_pair_step(nlse_ctx *c, double dt, int variant)
{
    Step3DArgs a;
    a.psin = c->psi;
    a.psi_out = c->psi2;
    a.K = c->K;
    a.B = c->B;
    a.V = c->V;
    for (int d = 0; d < 3; ++d) a.DB[d] = c->DB[d];
    a.L = c->L;
    a.c = base_coeffs(c->p);
    a.ck[0] = dt / 2.0;
    a.ck[1] = dt / 2.0;
    a.ck[2] = dt;
    a.ck[3] = dt / 6.0;
    a.variant = variant - stage3d_variants();
    hipError_t e = launch_step3d(c->prec, a, c->stream);
    if (e == hipSuccess) std::swap(c->psi, c->psi2);
    return e;
}

// One RK4 step of a 2D context with a whole-step variant: psi -> psi2, then swap.
static hipError_t launch_whole_step(nlse_ctx *c, double dt, int variant)
{
    Step2DArgs a;
    a.psi_in = c->psi;
    a.psi_out = c->psi2;
    a.V = c->V ? c->V : c->V0;
    a.DB[0] = c->DB[0];
    a.DB[1] = c->DB[1];
    a.L = c->L;
    a.c = base_coeffs(c->p);
    a.ck[0] = dt / 2.0;
    a.ck[1] = dt / 2.0;
    a.ck[2] = dt;
    a.ck[3] = dt / 6.0;
    a.variant = variant - stage2d_variants();
    a.stencil = c->stencil;
    a.msd = c->p.bc == NLSE_BC_MSD;
    hipError_t e = launch_step2d(c->prec, a, c->stream);
    if (e == hipSuccess) std::swap(c->psi, c->psi2);
    return e;
}

// One RK4 step with the given variant.
// A 1D context: `nsteps` RK4 steps in one launch of the on-chip solver.
static hipError_t launch_1d(nlse_ctx *c, double dt, int64_t nsteps, int variant)
{
    Solve1DArgs a;
    a.psin = c->psi;
    a.V = c->V;
    a.L = c->L;
    a.c = base_coeffs(c->p);
    a.k = dt;
    a.k2 = dt / 2.0;
    a.k6 = dt / 6.0;
    a.nsteps = nsteps;
    a.msd = c->p.bc == NLSE_BC_MSD;
    a.variant = variant;
    a.stencil = c->stencil;
    return launch_solve1d(c->prec, a, c->stream);
}

static hipError_t launch_rk4_step(nlse_ctx *c, double dt, int variant)
{
    if (c->p.ndim == 1) return launch_1d(c, dt, 1, variant);
    if (whole_step(c, variant)) return c->p.ndim == 2 ? launch_whole_step(c, dt, variant) : launch_pair_step(c, dt, variant);
    for (int st = 1; st <= 4; ++st) {
        hipError_t e = launch_stage(c, st, dt, variant);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

extern "C" {

const char *nlse_last_error(void) { return g_err.c_str(); }

int nlse_variant_count(const nlse_ctx *c)
{
    if (!c) return fail(NLSE_E_INVAL, "NULL context");
    return variant_count(c);
}

int nlse_set_variant(nlse_ctx *c, int variant)
{
    if (!c) return fail(NLSE_E_INVAL, "NULL context");
    if (variant < 0 || variant >= variant_count(c)) return fail(NLSE_E_INVAL, "variant out of range");
    c->variant = variant;
    return NLSE_OK;
}

int nlse_get_variant(const nlse_ctx *c)
{
    if (!c) return fail(NLSE_E_INVAL, "NULL context");
    return c->variant;
}

int nlse_set_stencil(nlse_ctx *c, int32_t stencil)
{
    if (!c) return fail(NLSE_E_INVAL, "NULL context");
    if (stencil < NLSE_STENCIL_2SHOC || stencil > NLSE_STENCIL_CD) return fail(NLSE_E_INVAL, "unknown stencil");
    if (stencil != NLSE_STENCIL_2SHOC && c->p.bc != NLSE_BC_DIRICHLET)
        return fail(NLSE_E_UNSUPPORTED, "the alternative stencils are implemented for Dirichlet boundaries only");
    c->stencil = stencil;
    if (c->variant >= variant_count(c)) c->variant = 0;   // the 3D two-stage variants are 2SHOC only
    return NLSE_OK;
}

int nlse_get_stencil(const nlse_ctx *c)
{
    if (!c) return fail(NLSE_E_INVAL, "NULL context");
    return c->stencil;
}

int nlse_autotune(nlse_ctx *c, int reps, int force, int *chosen)
{
    if (!c) return fail(NLSE_E_INVAL, "NULL context");
    if (!c->have_field) return fail(NLSE_E_INVAL, "no field set");
    if (reps < 1) reps = 1;
    const int nv = variant_count(c);
    if (nv > 1) {
        {
            std::lock_guard<std::mutex> g(g_tuned_mu);
            auto it = g_tuned.find(tune_key(c));
            if (!force && it != g_tuned.end() && it->second < nv) {
                c->variant = it->second;
                if (chosen) *chosen = c->variant;
                return NLSE_OK;
            }
        }
        // Time `reps` whole RK4 steps of every variant (twice, keeping the fastest) on a
        // copy of the field, then put the field back: the integration state is unchanged.
        const double dt = 0.5 * c->kmax;
        const size_t bytes = (size_t)c->L.total * c->esM;
        void *save = nullptr;
        if (hipMalloc(&save, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(NLSE_E_NOMEM, "autotune: no memory for the field copy");
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float best = 1e30f;
        int bestv = 0;
        hipError_t e = hipMemcpyAsync(save, c->psi, bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        for (int round = 0; round < 2 && e == hipSuccess; ++round) {
            for (int v = 0; v < nv && e == hipSuccess; ++v) {
                e = launch_rk4_step(c, dt, v);   // warm
                if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
                if (c->p.ndim == 1 && e == hipSuccess) e = launch_1d(c, dt, 16 * (int64_t)reps, v);   // one launch
                for (int r = 0; r < reps && c->p.ndim > 1 && e == hipSuccess; ++r) e = launch_rk4_step(c, dt, v);
                if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && ms < best) {
                    best = ms;
                    bestv = v;
                }
            }
        }
        if (e == hipSuccess) e = hipMemcpyAsync(c->psi, save, bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(save);
        if (e != hipSuccess) return hipfail(e, "autotune");
        c->variant = bestv;
        std::lock_guard<std::mutex> g(g_tuned_mu);
        g_tuned[tune_key(c)] = bestv;
    }
    if (chosen) *chosen = c->variant;
    return NLSE_OK;
}

// Copy between a pitched device array (rows of `width` bytes, `dpitch` apart) and contiguous
// host memory, synchronously.  A pitched copy straight to or from pageable host memory has
// returned stale data when the HIP runtime was instrumented (a kernel tracer), so the host data
// goes through a contiguous device buffer: one linear host copy, one pitched device-to-device copy.
static hipError_t pitched_host_copy(void *dev, size_t dpitch, void *host, size_t width, int64_t rows, bool to_dev,
                                   hipStream_t st)
{
    const size_t bytes = width * (size_t)rows;
    void *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, bytes);
    if (e != hipSuccess) return e;
    if (to_dev) {
        e = hipMemcpyAsync(tmp, host, bytes, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpy2DAsync(dev, dpitch, tmp, width, width, rows, hipMemcpyDeviceToDevice, st);
    } else {
        e = hipMemcpy2DAsync(tmp, width, dev, dpitch, width, rows, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(host, tmp, bytes, hipMemcpyDeviceToHost, st);
    }
    const hipError_t es = hipStreamSynchronize(st);
    if (e == hipSuccess) e = es;
    (void)hipFree(tmp);
    return e;
}

int nlse_create(nlse_ctx **out, const nlse_params *p)
{
    if (!out || !p) return fail(NLSE_E_INVAL, "nlse_create: NULL argument");
    *out = nullptr;
    if (p->ndim < 1 || p->ndim > 3) return fail(NLSE_E_INVAL, "ndim must be 1, 2 or 3");
    for (int a = 0; a < p->ndim; ++a)
        if (p->n[a] < 2) return fail(NLSE_E_INVAL, "n[a] must be >= 2 intervals");
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return fail(NLSE_E_INVAL, "h must be > 0");
    if (!(p->a > 0.0) || !std::isfinite(p->a)) return fail(NLSE_E_INVAL, "a must be > 0");
    if (!std::isfinite(p->s)) return fail(NLSE_E_INVAL, "s must be finite");
    if (p->bc != NLSE_BC_DIRICHLET && p->bc != NLSE_BC_MSD) return fail(NLSE_E_INVAL, "unknown bc");
    if (p->prec != NLSE_F64 && p->prec != NLSE_F32 && p->prec != NLSE_F32_MIXED)
        return fail(NLSE_E_INVAL, "unknown precision");
    if (p->bc == NLSE_BC_MSD && p->ndim == 1 && p->n[0] < 4) return fail(NLSE_E_INVAL, "MSD needs n >= 4 intervals");
    double padded = 1.0;   // an upper bound of the padded element count, without integer overflow
    for (int a = 0; a < p->ndim; ++a) padded *= (double)p->n[a] + 128.0;
    if (padded > 0x1p50) return fail(NLSE_E_NOMEM, "field too large for any device");

    nlse_ctx *c = new nlse_ctx();
    c->p = *p;
    c->p.V = nullptr;
    c->L = make_layout(p->ndim, p->n);
    c->prec = (Prec)p->prec;
    c->esR = c->prec == P_F64 ? 16 : 8;
    c->esM = c->prec == P_F32 ? 8 : 16;
    c->rR = c->esR / 2;
    c->stream = (hipStream_t)p->stream;
    if (p->ndim == 1 && c->L.nx + 1 > solve1d_max_nodes(c->prec)) {
        free_ctx(c);
        return fail(NLSE_E_UNSUPPORTED, "1D field larger than the on-chip solver holds");
    }
    if (p->ndim == 3 && c->L.total >= (int64_t(1) << 31)) {   // the 3D kernels' 32-bit element offsets
        free_ctx(c);
        return fail(NLSE_E_UNSUPPORTED, "3D field of 2^31 or more padded elements");
    }

    const size_t T = (size_t)c->L.total;
    auto alloc = [&](void **ptr, size_t bytes) -> int {
        hipError_t e = hipMalloc(ptr, bytes);
        if (e != hipSuccess) return fail(NLSE_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        e = hipMemset(*ptr, 0, bytes);
        if (e != hipSuccess) return hipfail(e, "hipMemset");
        return NLSE_OK;
    };
    int rc = alloc(&c->psi, T * c->esM);
    if (!rc && (p->ndim == 2 || step3d_ok(c))) rc = alloc(&c->psi2, T * c->esM);
    if (!rc && p->ndim > 1) rc = alloc(&c->A, T * c->esR);
    if (!rc && p->ndim > 1) rc = alloc(&c->B, T * c->esR);
    if (!rc && p->ndim > 1) rc = alloc(&c->K, T * c->esR);
    for (int a = 0; a < p->ndim && !rc; ++a) rc = alloc(&c->DB[a], 2 * (size_t)face_nodes(c->L, a) * c->esR);
    if (!rc) rc = alloc((void **)&c->red, (2 * (size_t)reduce_partials() + 4) * sizeof(double));
    if (!rc && p->V) {
        rc = alloc(&c->V, T * c->rR);
        if (!rc) {
            // convert to the stage precision and scatter rows into the padded layout
            const int64_t rows = c->L.py * (c->L.nz + 1), w = c->L.nx + 1;
            std::vector<unsigned char> host((size_t)rows * w * c->rR);
            for (int64_t i = 0; i < rows * w; ++i) {
                if (c->rR == 8) ((double *)host.data())[i] = p->V[i];
                else ((float *)host.data())[i] = (float)p->V[i];
            }
            hipError_t e = pitched_host_copy((char *)c->V + c->L.ox * c->rR, c->L.px * c->rR, host.data(),
                                             w * c->rR, rows, true, c->stream);
            if (e != hipSuccess) rc = hipfail(e, "copy of V");
        }
    }
    if (!rc && p->ndim == 2 && !p->V) rc = alloc(&c->V0, T * c->rR);   // alloc zero-fills
    if (rc) {
        free_ctx(c);
        return rc;
    }
    *out = c;
    return NLSE_OK;
}

void nlse_destroy(nlse_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
}

int nlse_launches_per_step(const nlse_ctx *c)
{
    if (!c) return fail(NLSE_E_INVAL, "NULL context");
    if (c->p.ndim == 1) return 0;
    if (whole_step(c, c->variant)) return c->p.ndim == 2 ? 1 : 2;
    return c->p.bc == NLSE_BC_MSD ? 8 : 4;   // MSD: boundary nodes and face values, then the interior, per stage
}

int nlse_sync(nlse_ctx *c)
{
    if (!c) return fail(NLSE_E_INVAL, "NULL context");
    HIPTRY(hipStreamSynchronize(c->stream));
    return NLSE_OK;
}

static int copy_field(nlse_ctx *c, void *dev_field, void *user, int on_device, bool to_dev)
{
    const Layout &L = c->L;
    const size_t es = c->esM;
    const int64_t rows = L.py * (L.nz + 1), w = L.nx + 1;
    char *dev = (char *)dev_field + L.ox * es;
    if (!on_device) {
        HIPTRY(pitched_host_copy(dev, L.px * es, user, w * es, rows, to_dev, c->stream));
    } else if (to_dev) {
        HIPTRY(hipMemcpy2DAsync(dev, L.px * es, user, w * es, w * es, rows, hipMemcpyDeviceToDevice, c->stream));
    } else {
        HIPTRY(hipMemcpy2DAsync(user, w * es, dev, L.px * es, w * es, rows, hipMemcpyDeviceToDevice, c->stream));
    }
    return NLSE_OK;
}

static int read_scalars(nlse_ctx *c, double *dst, int count)
{
    HIPTRY(hipMemcpyAsync(dst, c->red + 2 * reduce_partials(), count * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIPTRY(hipStreamSynchronize(c->stream));
    return NLSE_OK;
}

int nlse_max_dt(nlse_ctx *c, double *out)
{
    if (!c || !out) return fail(NLSE_E_INVAL, "nlse_max_dt: NULL argument");
    HIPTRY(launch_minmax_nonlin(c->prec, c->psi, c->V, c->L, c->p.s, c->red, c->red + 2 * reduce_partials(),
                                c->stream));
    double mm[2];
    int rc = read_scalars(c, mm, 2);
    if (rc) return rc;
    if (!std::isfinite(mm[0]) || !std::isfinite(mm[1])) return fail(NLSE_E_NONFINITE, "field is not finite");
    static const double gmax[3] = {64.0 / 12.0, 128.0 / 12.0, 192.0 / 12.0};
    static const double gmin[3] = {-4.0 / 12.0, -8.0 / 12.0, -12.0 / 12.0};
    const double h2a = c->p.h * c->p.h / c->p.a;
    const double lmin = h2a * mm[0], lmax = h2a * mm[1];
    double m = std::fmax(gmax[c->p.ndim - 1] - lmin, lmax - gmin[c->p.ndim - 1]);
    if (c->p.bc == NLSE_BC_MSD && c->p.ndim > 1) {
        Coeffs co = base_coeffs(c->p);
        const void *db[3] = {c->DB[0], c->DB[1], c->DB[2]};
        HIPTRY(launch_msd_faces(c->prec, true, c->psi, c->V, c->L, co, c->DB, c->stream));
        HIPTRY(launch_msd_bound(c->prec, c->psi, c->V, db, c->L, co, h2a, c->red + 2 * reduce_partials(), c->stream));
        double B;
        rc = read_scalars(c, &B, 1);
        if (rc) return rc;
        m = std::fmax(m, B);
    } else if (c->p.bc == NLSE_BC_MSD) {   // 1D: the two ends on the device
        HIPTRY(launch_edges1d(c->prec, c->psi, c->V, c->L, base_coeffs(c->p), true, h2a, c->DB[0],
                              c->red + 2 * reduce_partials(), c->stream));
        double B;
        rc = read_scalars(c, &B, 1);
        if (rc) return rc;
        m = std::fmax(m, B);
    }
    *out = std::sqrt(8.0) * c->p.h * c->p.h / (c->p.a * m);
    return NLSE_OK;
}

int nlse_set_field(nlse_ctx *c, const void *psi, int on_device)
{
    if (!c || !psi) return fail(NLSE_E_INVAL, "nlse_set_field: NULL argument");
    int rc = copy_field(c, c->psi, (void *)psi, on_device, true);
    if (rc) return rc;
    if (c->psi2)   // the whole-step / pair kernels write interiors only: give psi2 the boundary values
        HIPTRY(hipMemcpyAsync(c->psi2, c->psi, (size_t)c->L.total * c->esM, hipMemcpyDeviceToDevice, c->stream));
    if (c->p.ndim > 1) {
        HIPTRY(launch_master_to_stage(c->prec, c->psi, c->A, c->L, c->stream));
        HIPTRY(launch_master_to_stage(c->prec, c->psi, c->B, c->L, c->stream));
        Coeffs co = base_coeffs(c->p);   // Dirichlet face values are constants; MSD ones follow each stage
        if (c->p.bc == NLSE_BC_DIRICHLET) HIPTRY(launch_boundary_d(c->prec, c->psi, c->V, c->L, co, c->DB, c->stream));
    }
    c->have_field = true;
    double k;
    rc = nlse_max_dt(c, &k);
    if (rc) return rc;
    c->kmax = k;
    return NLSE_OK;
}

int nlse_get_field(nlse_ctx *c, void *out, int on_device)
{
    if (!c || !out) return fail(NLSE_E_INVAL, "nlse_get_field: NULL argument");
    return copy_field(c, c->psi, out, on_device, false);
}

int nlse_step(nlse_ctx *c, int64_t nsteps, double dt)
{
    if (!c) return fail(NLSE_E_INVAL, "NULL context");
    if (nsteps < 0) return fail(NLSE_E_INVAL, "nsteps must be >= 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(NLSE_E_INVAL, "dt must be > 0");
    if (!c->have_field) return fail(NLSE_E_INVAL, "no field set");
    if (!c->p.allow_unstable && dt > c->kmax) {
        char buf[160];
        snprintf(buf, sizeof buf, "dt = %.17g exceeds the stability bound %.17g", dt, c->kmax);
        return fail(NLSE_E_DT_UNSTABLE, buf);
    }
    if (nsteps == 0) return NLSE_OK;
    if (c->p.ndim == 1) {
        HIPTRY(launch_1d(c, dt, nsteps, c->variant));
        return NLSE_OK;
    }
    for (int64_t step = 0; step < nsteps; ++step) {
        hipError_t e = launch_rk4_step(c, dt, c->variant);
        if (e != hipSuccess) return hipfail(e, "RK4 step launch");
    }
    return NLSE_OK;
}

int nlse_mass(nlse_ctx *c, double *out)
{
    if (!c || !out) return fail(NLSE_E_INVAL, "nlse_mass: NULL argument");
    HIPTRY(launch_mass(c->prec, c->psi, c->L, c->red, c->red + 2 * reduce_partials(), c->stream));
    double m;
    int rc = read_scalars(c, &m, 1);
    if (rc) return rc;
    *out = std::pow(c->p.h, c->p.ndim) * m;
    if (!std::isfinite(*out)) return fail(NLSE_E_NONFINITE, "mass is not finite");
    return NLSE_OK;
}

int nlse_energy(nlse_ctx *c, double *out)
{
    if (!c || !out) return fail(NLSE_E_INVAL, "nlse_energy: NULL argument");
    Coeffs co = base_coeffs(c->p);
    if (c->p.ndim == 1)   // boundary closure of the current field (Eq. dbc_lap or Eq. msdbc_lap)
        HIPTRY(launch_edges1d(c->prec, c->psi, c->V, c->L, co, c->p.bc == NLSE_BC_MSD, 0.0, c->DB[0], nullptr,
                              c->stream));
    if (c->p.ndim > 1 && c->p.bc == NLSE_BC_MSD)   // face values of the current field (Eq. msdbc_lap)
        HIPTRY(launch_msd_faces(c->prec, true, c->psi, c->V, c->L, co, c->DB, c->stream));
    const void *db[3] = {c->DB[0], c->DB[1], c->DB[2]};
    HIPTRY(launch_energy(c->prec, c->psi, c->V, db, c->L, co, c->red, c->red + 2 * reduce_partials(), c->stream));
    double e;
    int rc = read_scalars(c, &e, 1);
    if (rc) return rc;
    *out = e;
    if (!std::isfinite(e)) return fail(NLSE_E_NONFINITE, "energy is not finite");
    return NLSE_OK;
}

}  // extern "C"
