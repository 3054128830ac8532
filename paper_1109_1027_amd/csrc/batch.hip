// Batched 2SHOC-RK4: thousands of independent 1D and 2D problems of uneven size
// advanced by one graph launch: a queue reset and two persistent kernels, captured
// once in a hipGraph.
//
// Each instance is an ordinary context (its own padded arrays, boundary closure,
// step-size bound); the batch adds a device table of instances, two work queues
// and the graph.  Workgroups of each persistent kernel pop instance indices from
// their queue (longest first) and advance the popped instance through all
// requested steps before popping again:
//   - 2D kernel: an instance advances by whole RK4 steps (wave2d.h); the waves of
//     the workgroup (12 in FP32, three per SIMD at the body's ~170 VGPRs, else 8) share out
//     its (strip, row segment) tasks, reading Psi^n and V and writing Psi^{n+1}
//     into the instance's second master buffer, one workgroup barrier per step; an
//     odd step count ends with a copy back;
//   - 1D kernel: an instance runs entirely on chip (onchip1d.h): HBM is touched
//     twice.
// Every workgroup leaves its loop when its queue is exhausted, so both grids
// always drain.  Instances never share memory, so no cross-workgroup
// synchronisation exists.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "ctx.h"
#include "onchip1d.h"
#include "wave2d.h"

using namespace nlse;

namespace nlse {

struct BatchItem {
    Layout L;
    void *psi, *psi2;
    const void *V;      // 2D: never nullptr (zeros when V = 0)
    const void *DB[2];
    Coeffs c;
    double dt;
    int msd;
};

// 1D workgroups: threads x nodes per thread.  FP32 fits 9 nodes per thread in 128 VGPRs,
// so 1024-thread workgroups run four waves per SIMD; the FP64-master types keep 512 threads.
template <typename R, typename M> struct Batch1D { static constexpr int BS = 512, NPT = 10; };
template <> struct Batch1D<float, float> { static constexpr int BS = 1024, NPT = 9; };
template <> struct Batch1D<float, double> { static constexpr int BS = 512, NPT = 17; };

// 2D workgroups: 12 waves in FP32, whose whole-step body needs about 170 VGPRs (three waves per
// SIMD; at 16 waves and 128 VGPRs it spills in the row loop), 8 waves otherwise.
template <typename R, typename M> struct Batch2DWaves { static constexpr int v = 8; };
template <> struct Batch2DWaves<float, float> { static constexpr int v = 12; };

__global__ void batch_reset_kernel(int *queue)
{
    if (threadIdx.x < 2) queue[threadIdx.x] = 0;
}

// Persistent kernel for the 2D instances (order[0 .. n2d)).
template <typename R, typename M, int Q, int NW>
__global__ __launch_bounds__(64 * NW) void batch2d_kernel(const BatchItem *items, const int *order, int n2d,
                                                          int *queue, int64_t nsteps)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];   // after s_item: keep 16-byte alignment
    __shared__ int s_item;
    auto *stg = reinterpret_cast<wave2d::Staging<R, Q> *>(smem);   // [NW], one per wave
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: item fields go to SGPRs
        if (it >= n2d) break;   // workgroup-uniform: the queue is exhausted
        const BatchItem &I = items[order[it]];
        const double dt = I.dt;
        const int strips = wave2d::strips(I.L.nx);
        const int tasks = strips * wave2d::segments<Q>(I.L.ny);
        Step2DArgs a;
        a.V = I.V;
        a.DB[0] = I.DB[0];
        a.DB[1] = I.DB[1];
        a.L = I.L;
        a.c = I.c;
        a.ck[0] = dt / 2.0;
        a.ck[1] = dt / 2.0;
        a.ck[2] = dt;
        a.ck[3] = dt / 6.0;
        a.variant = 0;
        a.stencil = 0;
        a.msd = 0;
        void *cur = I.psi, *nxt = I.psi2;
        for (int64_t step = 0; step < nsteps; ++step) {
            a.psi_in = cur;
            a.psi_out = nxt;
            for (int task = wv; task < tasks; task += NW)
                wave2d::step2d_wave<R, M, Q>(a, task % strips, task / strips, threadIdx.x & 63, stg[wv]);
            __syncthreads();   // Psi^{n+1} complete before any task reads it
            void *t = cur;
            cur = nxt;
            nxt = t;
        }
        if (cur != I.psi) {    // odd step count: the result is in psi2
            const C<M> *src = (const C<M> *)cur;
            C<M> *dst = (C<M> *)I.psi;
            for (int64_t e = threadIdx.x; e < I.L.total; e += 64 * NW) dst[e] = src[e];
        }
    }
}

// Persistent kernel for the 1D instances (order[n2d .. n2d + n1d)).
template <typename R, typename M, int BS, int NPT>
__global__ __launch_bounds__(BS) void batch1d_kernel(const BatchItem *items, const int *order, int n1d,
                                                           int *queue, int64_t nsteps)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];   // after s_item: keep 16-byte alignment
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: item fields go to SGPRs
        if (it >= n1d) break;
        const BatchItem &I = items[order[it]];
        Solve1DArgs a;
        a.psin = I.psi;
        a.V = I.V;
        a.L = I.L;
        a.c = I.c;
        a.k = I.dt;
        a.k2 = I.dt / 2.0;
        a.k6 = I.dt / 6.0;
        a.nsteps = nsteps;
        a.msd = I.msd;
        a.variant = 0;
        a.stencil = 0;
        // The solver body with the smallest node bound that holds the instance: every slot
        // of its register arrays costs instructions whether used or not.
        const int npt = max(3, (int)((I.L.nx + 1 + BS - 1) / BS));
        if (npt <= 3) {
            solve1d_onchip<R, M, BS, 3>(a, smem);
        } else if (npt <= 5) {
            if constexpr (NPT > 5) solve1d_onchip<R, M, BS, 5>(a, smem);
            else solve1d_onchip<R, M, BS, NPT>(a, smem);
        } else if (npt <= 7) {
            if constexpr (NPT > 7) solve1d_onchip<R, M, BS, 7>(a, smem);
            else solve1d_onchip<R, M, BS, NPT>(a, smem);
        } else {
            solve1d_onchip<R, M, BS, NPT>(a, smem);
        }
    }
}

// Variant v selects the row-segment length of the 2D whole-step tasks: 56, 29 or 20 rows.
constexpr int BATCH_VARIANTS = 3;

struct BatchLaunch {
    const BatchItem *items;
    const int *order;        // the n2d 2D instances, then the n1d 1D instances (longest first)
    int n2d, n1d;
    int *queue;              // [2]: next 2D, next 1D
    int64_t nsteps;
    int grid2d, grid1d;
};

template <typename R, typename M, int Q>
static hipError_t launch_batch_q(const BatchLaunch &L, hipStream_t st)
{
    constexpr int NW = Batch2DWaves<R, M>::v;
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, L.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (L.n2d > 0) {
        const size_t lds = sizeof(wave2d::Staging<R, Q>) * NW;
        hipLaunchKernelGGL((batch2d_kernel<R, M, Q, NW>), dim3(L.grid2d), dim3(64 * NW), lds, st, L.items, L.order,
                           L.n2d, L.queue, L.nsteps);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (L.n1d > 0) {
        constexpr int BS = Batch1D<R, M>::BS;
        const size_t lds1 = onchip1d_lds<R, BS>();
        hipLaunchKernelGGL((batch1d_kernel<R, M, BS, Batch1D<R, M>::NPT>), dim3(L.grid1d), dim3(BS), lds1, st,
                           L.items, L.order + L.n2d, L.n1d, L.queue + 1, L.nsteps);
        e = hipGetLastError();
    }
    return e;
}

template <typename R, typename M>
static hipError_t launch_batch_v(int variant, const BatchLaunch &L, hipStream_t st)
{
    switch (variant) {
    case 0: return launch_batch_q<R, M, 8>(L, st);
    case 1: return launch_batch_q<R, M, 5>(L, st);
    case 2: return launch_batch_q<R, M, 4>(L, st);
    default: return hipErrorInvalidValue;
    }
}

static hipError_t launch_batch(Prec prec, int variant, const BatchLaunch &L, hipStream_t st)
{
    switch (prec) {
    case P_F64: return launch_batch_v<double, double>(variant, L, st);
    case P_F32: return launch_batch_v<float, float>(variant, L, st);
    default: return launch_batch_v<float, double>(variant, L, st);
    }
}

}  // namespace nlse

struct nlse_batch {
    std::vector<nlse_ctx *> ctx;
    std::vector<double> dt;
    Prec prec;
    hipStream_t stream = nullptr;       // caller's stream (graph launches)
    hipStream_t cap = nullptr;          // private stream for graph capture
    BatchItem *d_items = nullptr;
    int *d_order = nullptr;
    int *d_queue = nullptr;
    bool dirty = true;
    int variant = 0;
    int n2d = 0, n1d = 0;       // instance counts by kind
    int cus = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t graph_steps = -1;
    int graph_variant = -1;
};

static void batch_free(nlse_batch *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (nlse_ctx *c : b->ctx) nlse_destroy(c);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_order) (void)hipFree(b->d_order);
    if (b->d_queue) (void)hipFree(b->d_queue);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

static int upload_items(nlse_batch *b)
{
    const int n = (int)b->ctx.size();
    std::vector<BatchItem> items(n);
    std::vector<int64_t> work(n);
    for (int i = 0; i < n; ++i) {
        nlse_ctx *c = b->ctx[i];
        BatchItem &it = items[i];
        std::memset(&it, 0, sizeof it);
        it.L = c->L;
        it.psi = c->psi;
        it.psi2 = c->psi2;
        it.V = c->V ? c->V : c->V0;
        it.DB[0] = c->DB[0];
        it.DB[1] = c->DB[1];
        it.c = base_coeffs(c->p);
        it.dt = b->dt[i];
        it.msd = c->p.bc == NLSE_BC_MSD;
        // order: the 2D instances first (their kernel runs first), then the 1D ones, each kind
        // longest first
        work[i] = c->p.ndim == 2 ? (int64_t(1) << 40) + (c->L.nx + 1) * (c->L.ny + 1) : (c->L.nx + 1);
    }
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    HIPTRY(hipMemcpyAsync(b->d_items, items.data(), sizeof(BatchItem) * n, hipMemcpyHostToDevice, b->stream));
    HIPTRY(hipMemcpyAsync(b->d_order, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, b->stream));
    HIPTRY(hipStreamSynchronize(b->stream));
    b->dirty = false;
    return NLSE_OK;
}

extern "C" {

int nlse_batch_create(nlse_batch **out, const nlse_params *items, int32_t count)
{
    if (!out || !items || count <= 0) return fail(NLSE_E_INVAL, "nlse_batch_create: bad arguments");
    *out = nullptr;
    for (int i = 0; i < count; ++i) {
        if (items[i].ndim != 1 && items[i].ndim != 2)
            return fail(NLSE_E_UNSUPPORTED, "batched instances are 1D or 2D");
        if (items[i].ndim == 2 && items[i].bc != NLSE_BC_DIRICHLET)
            return fail(NLSE_E_UNSUPPORTED, "batched 2D instances take the Dirichlet boundary");
        if (items[i].prec != items[0].prec) return fail(NLSE_E_INVAL, "all instances need the same precision");
        if (items[i].stream != items[0].stream) return fail(NLSE_E_INVAL, "all instances need the same stream");
    }
    nlse_batch *b = new nlse_batch();
    b->prec = (Prec)items[0].prec;
    b->stream = (hipStream_t)items[0].stream;
    const int64_t cap1d = b->prec == P_F64   ? (int64_t)Batch1D<double, double>::BS * Batch1D<double, double>::NPT
                          : b->prec == P_F32 ? (int64_t)Batch1D<float, float>::BS * Batch1D<float, float>::NPT
                                             : (int64_t)Batch1D<float, double>::BS * Batch1D<float, double>::NPT;
    for (int i = 0; i < count; ++i) {
        if (items[i].ndim == 1 && items[i].n[0] + 1 > cap1d) {
            batch_free(b);
            return fail(NLSE_E_UNSUPPORTED, "1D instance larger than one workgroup holds");
        }
        nlse_ctx *c = nullptr;
        int rc = nlse_create(&c, &items[i]);
        if (rc) {
            batch_free(b);
            return rc;
        }
        if (items[i].ndim == 2 && c->L.total >= (int64_t(1) << 31)) {   // 32-bit offsets in wave2d.h
            nlse_destroy(c);
            batch_free(b);
            return fail(NLSE_E_UNSUPPORTED, "2D instance too large for the batched launch");
        }
        b->ctx.push_back(c);
        b->dt.push_back(0.0);
        if (items[i].ndim == 1) ++b->n1d;
        else ++b->n2d;
    }
    hipError_t e = hipMalloc((void **)&b->d_items, sizeof(BatchItem) * count);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_order, sizeof(int) * count);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_queue, 2 * sizeof(int));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        batch_free(b);
        return fail(NLSE_E_NOMEM, std::string("batch allocation: ") + hipGetErrorString(e));
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->cus = cus > 0 ? cus : 256;
    *out = b;
    return NLSE_OK;
}

void nlse_batch_destroy(nlse_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
}

int32_t nlse_batch_count(const nlse_batch *b) { return b ? (int32_t)b->ctx.size() : 0; }

static int check_item(const nlse_batch *b, int32_t i)
{
    if (!b) return fail(NLSE_E_INVAL, "NULL batch");
    if (i < 0 || i >= (int32_t)b->ctx.size()) return fail(NLSE_E_INVAL, "instance index out of range");
    return NLSE_OK;
}

int nlse_batch_set_field(nlse_batch *b, int32_t i, const void *psi, int on_device)
{
    int rc = check_item(b, i);
    if (rc) return rc;
    rc = nlse_set_field(b->ctx[i], psi, on_device);
    if (rc) return rc;
    b->dirty = true;
    return NLSE_OK;
}

int nlse_batch_get_field(nlse_batch *b, int32_t i, void *out, int on_device)
{
    int rc = check_item(b, i);
    return rc ? rc : nlse_get_field(b->ctx[i], out, on_device);
}

int nlse_batch_max_dt(nlse_batch *b, int32_t i, double *out)
{
    int rc = check_item(b, i);
    return rc ? rc : nlse_max_dt(b->ctx[i], out);
}

int nlse_batch_mass(nlse_batch *b, int32_t i, double *out)
{
    int rc = check_item(b, i);
    return rc ? rc : nlse_mass(b->ctx[i], out);
}

int nlse_batch_set_dt(nlse_batch *b, int32_t i, double dt)
{
    int rc = check_item(b, i);
    if (rc) return rc;
    nlse_ctx *c = b->ctx[i];
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(NLSE_E_INVAL, "dt must be > 0");
    if (!c->have_field) return fail(NLSE_E_INVAL, "set the instance's field before its dt");
    if (!c->p.allow_unstable && dt > c->kmax) return fail(NLSE_E_DT_UNSTABLE, "dt exceeds the instance's bound");
    b->dt[i] = dt;
    b->dirty = true;
    return NLSE_OK;
}

int nlse_batch_variant_count(const nlse_batch *b) { return b ? BATCH_VARIANTS : fail(NLSE_E_INVAL, "NULL batch"); }

int nlse_batch_set_variant(nlse_batch *b, int variant)
{
    if (!b) return fail(NLSE_E_INVAL, "NULL batch");
    if (variant < 0 || variant >= BATCH_VARIANTS) return fail(NLSE_E_INVAL, "variant out of range");
    b->variant = variant;
    return NLSE_OK;
}

int nlse_batch_get_variant(const nlse_batch *b) { return b ? b->variant : fail(NLSE_E_INVAL, "NULL batch"); }

int nlse_batch_step(nlse_batch *b, int64_t nsteps)
{
    if (!b) return fail(NLSE_E_INVAL, "NULL batch");
    if (nsteps < 0) return fail(NLSE_E_INVAL, "nsteps must be >= 0");
    for (size_t i = 0; i < b->ctx.size(); ++i)
        if (!(b->dt[i] > 0.0)) return fail(NLSE_E_INVAL, "every instance needs a field and a dt");
    if (nsteps == 0) return NLSE_OK;
    if (b->dirty) {
        int rc = upload_items(b);
        if (rc) return rc;
    }
    if (!b->exec || b->graph_steps != nsteps || b->graph_variant != b->variant) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        HIPTRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
        BatchLaunch L;
        L.items = b->d_items;
        L.order = b->d_order;
        L.n2d = b->n2d;
        L.n1d = b->n1d;
        L.queue = b->d_queue;
        L.nsteps = nsteps;
        L.grid2d = std::max(1, std::min(b->n2d, b->cus));
        L.grid1d = std::max(1, std::min(b->n1d, b->cus));
        hipError_t e = launch_batch(b->prec, b->variant, L, b->cap);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap, &g);
        if (e != hipSuccess) return hipfail(e, "batch kernel capture");
        if (e2 != hipSuccess) return hipfail(e2, "hipStreamEndCapture");
        b->graph = g;
        HIPTRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_steps = nsteps;
        b->graph_variant = b->variant;
    }
    HIPTRY(hipGraphLaunch(b->exec, b->stream));
    return NLSE_OK;
}

// Autotuner of the batched launch: for every variant, one untimed call of `nsteps` steps
// (item upload, graph capture and instantiation, first launch), then the fastest of three
// timed calls of the same graph (events around the graph launch only); keeps the fastest
// variant.  The masters Psi^n of all instances are saved before and restored after each
// call (device-to-device), so the integration state is unchanged.
int nlse_batch_autotune(nlse_batch *b, int64_t nsteps, int force, int *chosen)
{
    if (!b) return fail(NLSE_E_INVAL, "NULL batch");
    if (nsteps < 1) nsteps = 1;
    if (b->graph_variant >= 0 && !force) {
        if (chosen) *chosen = b->variant;
        return NLSE_OK;
    }
    size_t total = 0;
    std::vector<size_t> off(b->ctx.size());
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        off[i] = total;
        total += ((b->ctx[i]->L.total * b->ctx[i]->esM + 255) / 256) * 256;
    }
    void *save = nullptr;
    HIPTRY(hipMalloc(&save, total));
    auto copy_all = [&](bool to_save) -> hipError_t {
        for (size_t i = 0; i < b->ctx.size(); ++i) {
            nlse_ctx *c = b->ctx[i];
            char *s = (char *)save + off[i];
            hipError_t e = hipMemcpyAsync(to_save ? (void *)s : c->psi, to_save ? c->psi : (void *)s,
                                          c->L.total * c->esM, hipMemcpyDeviceToDevice, b->stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipEvent_t e0, e1;
    int rc = NLSE_OK;
    float best = 1e30f;
    int bestv = b->variant;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(save);
        return fail(NLSE_E_HIP, "hipEventCreate");
    }
    hipError_t he = copy_all(true);
    for (int v = 0; v < BATCH_VARIANTS && he == hipSuccess && !rc; ++v) {
        b->variant = v;
        rc = nlse_batch_step(b, nsteps);   // untimed: upload, capture, instantiate, first launch
        if (!rc) he = copy_all(false);
        for (int rep = 0; rep < 3 && he == hipSuccess && !rc; ++rep) {
            he = hipEventRecord(e0, b->stream);
            if (he == hipSuccess) rc = nlse_batch_step(b, nsteps);   // the graph exists: launch only
            if (he == hipSuccess && !rc) he = hipEventRecord(e1, b->stream);
            if (he == hipSuccess && !rc) he = hipEventSynchronize(e1);
            float ms = 0;
            if (he == hipSuccess && !rc) he = hipEventElapsedTime(&ms, e0, e1);
            if (he == hipSuccess && !rc && ms < best) {
                best = ms;
                bestv = v;
            }
            if (he == hipSuccess) he = copy_all(false);
        }
    }
    (void)hipStreamSynchronize(b->stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(save);
    if (rc) return rc;
    if (he != hipSuccess) return hipfail(he, "batch autotune");
    b->variant = bestv;
    if (chosen) *chosen = bestv;
    return NLSE_OK;
}

int nlse_batch_sync(nlse_batch *b)
{
    if (!b) return fail(NLSE_E_INVAL, "NULL batch");
    HIPTRY(hipStreamSynchronize(b->stream));
    return NLSE_OK;
}

}  // extern "C"
