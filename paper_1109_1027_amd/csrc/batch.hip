// Batched 2SHOC-RK4: thousands of independent 1D and 2D problems of uneven size
// advanced by one persistent kernel, captured once in a hipGraph.
//
// Each instance is an ordinary context (its own padded arrays, boundary closure,
// step-size bound); the batch adds a device table of instances, a work queue
// and the graph.  Workgroups of the persistent kernel pop instance indices from
// the queue in longest-first order and advance the popped instance through all
// requested steps before popping again:
//   - a 1D instance runs entirely on chip (onchip1d.h): HBM is touched twice;
//   - a 2D instance is swept tile by tile by all waves of the workgroup
//     (tile2d.h), with a workgroup barrier between RK4 stages; its five arrays
//     stream through L2 / the Infinity Cache / HBM.
// Every workgroup leaves the loop when the queue is exhausted, so the grid
// always drains.  Instances never share memory, so no cross-workgroup
// synchronisation exists.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "ctx.h"
#include "onchip1d.h"
#include "tile2d.h"

using namespace nlse;

namespace nlse {

struct BatchItem {
    Layout L;
    void *psi, *A, *B, *K;
    const void *V;
    const void *DB[2];
    Coeffs c;
    double dt;
    int msd;
};

constexpr int BATCH_BS = 512;
constexpr int BATCH_NW = BATCH_BS / 64;

template <typename R> struct BatchNPT;
template <> struct BatchNPT<double> { static constexpr int v = 10; };
template <> struct BatchNPT<float> { static constexpr int v = 17; };

__global__ void batch_reset_kernel(int *queue)
{
    if (threadIdx.x == 0) queue[0] = 0;
}

template <typename R, typename M, int RW>
__global__ __launch_bounds__(BATCH_BS) void batch_kernel(const BatchItem *items, const int *order, int count,
                                                         int *queue, int64_t nsteps)
{
    extern __shared__ unsigned char smem[];
    __shared__ int s_item;
    constexpr int NPT = BatchNPT<R>::v;
    using Row = C<R>[RW][TILE_W + 4];
    using RowD = C<R>[RW][TILE_W + 2];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= count) break;   // workgroup-uniform: the queue is exhausted
        const BatchItem &I = items[order[it]];
        const double dt = I.dt;
        if (I.L.dim == 1) {
            Solve1DArgs a;
            a.psin = I.psi;
            a.V = I.V;
            a.L = I.L;
            a.c = I.c;
            a.k = dt;
            a.k2 = dt / 2.0;
            a.k6 = dt / 6.0;
            a.nsteps = nsteps;
            a.msd = I.msd;
            solve1d_onchip<R, M, BATCH_BS, NPT>(a, smem);
        } else {
            Row *lds = reinterpret_cast<Row *>(smem);
            RowD *ldx = reinterpret_cast<RowD *>(smem + sizeof(Row) * BATCH_NW);
            const int64_t tiles_x = (I.L.nx - 1 + TILE_W - 1) / TILE_W;
            const int64_t tiles = tiles_x * ((I.L.ny - 1 + RW - 1) / RW);
            const double ck[4] = {dt / 2.0, dt / 2.0, dt, dt / 6.0};
            void *ins[4] = {I.psi, I.A, I.B, I.A};
            void *outs[4] = {I.A, I.B, I.A, nullptr};
            const int wv = threadIdx.x >> 6;
            for (int64_t step = 0; step < nsteps; ++step) {
                for (int st = 0; st < 4; ++st) {
                    StageArgs a;
                    a.in = ins[st];
                    a.out = outs[st];
                    a.psin = I.psi;
                    a.K = I.K;
                    a.V = I.V;
                    a.DB[0] = I.DB[0];
                    a.DB[1] = I.DB[1];
                    a.DB[2] = nullptr;
                    a.L = I.L;
                    a.c = I.c;
                    a.c.ck = ck[st];
                    a.stage = st + 1;
                    a.variant = 0;
                    for (int64_t base = 0; base < tiles; base += BATCH_NW) {
                        if (st == 0)
                            stage2d_tile<M, R, M, RW, BATCH_NW>(a, base + wv, tiles_x, tiles, lds, ldx);
                        else
                            stage2d_tile<R, R, M, RW, BATCH_NW>(a, base + wv, tiles_x, tiles, lds, ldx);
                    }
                    __syncthreads();   // this stage's outputs are the next stage's inputs
                }
            }
        }
    }
}

template <typename R, typename M, int RW>
static size_t batch_lds(int64_t max1d_nodes, bool has2d)
{
    size_t l1 = 2 * sizeof(C<R>) * (size_t)max1d_nodes;
    size_t l2 = has2d ? sizeof(C<R>) * RW * (2 * TILE_W + 6) * BATCH_NW : 0;
    return std::max(l1, l2);
}

template <typename R, typename M, int RW>
static hipError_t launch_batch_rw(const BatchItem *items, const int *order, int count, int *queue, int64_t nsteps,
                                  int grid, size_t lds, hipStream_t st)
{
    (void)hipFuncSetAttribute((const void *)batch_kernel<R, M, RW>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, st, queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batch_kernel<R, M, RW>), dim3(grid), dim3(BATCH_BS), lds, st, items, order, count, queue,
                       nsteps);
    return hipGetLastError();
}

// Variant v selects the 2D tile height: (8, 4) rows per wave for FP32 / mixed,
// (4, 2) for FP64 (LDS holds 16 waves x RW rows x 134 complex values).
static size_t batch_lds_for(Prec prec, int variant, int64_t max1d, bool has2d)
{
    if (prec == P_F64) return variant == 0 ? batch_lds<double, double, 4>(max1d, has2d)
                                            : batch_lds<double, double, 2>(max1d, has2d);
    return variant == 0 ? batch_lds<float, float, 8>(max1d, has2d) : batch_lds<float, float, 4>(max1d, has2d);
}

static hipError_t launch_batch(Prec prec, int variant, const BatchItem *items, const int *order, int count,
                               int *queue, int64_t nsteps, int grid, size_t lds, hipStream_t st)
{
    switch (prec) {
    case P_F64:
        return variant == 0 ? launch_batch_rw<double, double, 4>(items, order, count, queue, nsteps, grid, lds, st)
                            : launch_batch_rw<double, double, 2>(items, order, count, queue, nsteps, grid, lds, st);
    case P_F32:
        return variant == 0 ? launch_batch_rw<float, float, 8>(items, order, count, queue, nsteps, grid, lds, st)
                            : launch_batch_rw<float, float, 4>(items, order, count, queue, nsteps, grid, lds, st);
    default:
        return variant == 0 ? launch_batch_rw<float, double, 8>(items, order, count, queue, nsteps, grid, lds, st)
                            : launch_batch_rw<float, double, 4>(items, order, count, queue, nsteps, grid, lds, st);
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
    int grid = 0;
    size_t lds = 0;
    int64_t max1d = 0;
    bool has2d = false;
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
        it.A = c->A;
        it.B = c->B;
        it.K = c->K;
        it.V = c->V;
        it.DB[0] = c->DB[0];
        it.DB[1] = c->DB[1];
        it.c = base_coeffs(c->p);
        it.dt = b->dt[i];
        it.msd = c->p.bc == NLSE_BC_MSD;
        // work estimate for longest-first ordering: 2D instances stream through memory
        work[i] = c->p.ndim == 1 ? (c->L.nx + 1) : 16 * (c->L.nx + 1) * (c->L.ny + 1);
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
        if (items[i].prec != items[0].prec) return fail(NLSE_E_INVAL, "all instances need the same precision");
        if (items[i].stream != items[0].stream) return fail(NLSE_E_INVAL, "all instances need the same stream");
    }
    nlse_batch *b = new nlse_batch();
    b->prec = (Prec)items[0].prec;
    b->stream = (hipStream_t)items[0].stream;
    const int64_t cap1d = b->prec == P_F64 ? (int64_t)BATCH_BS * BatchNPT<double>::v
                                           : (int64_t)BATCH_BS * BatchNPT<float>::v;
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
        b->ctx.push_back(c);
        b->dt.push_back(0.0);
        if (items[i].ndim == 1) b->max1d = std::max(b->max1d, items[i].n[0] + 1);
        else b->has2d = true;
    }
    hipError_t e = hipMalloc((void **)&b->d_items, sizeof(BatchItem) * count);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_order, sizeof(int) * count);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_queue, sizeof(int));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        batch_free(b);
        return fail(NLSE_E_NOMEM, std::string("batch allocation: ") + hipGetErrorString(e));
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->grid = std::max(1, std::min(count, cus > 0 ? cus : 256));
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

int nlse_batch_variant_count(const nlse_batch *b) { return b ? 2 : fail(NLSE_E_INVAL, "NULL batch"); }

int nlse_batch_set_variant(nlse_batch *b, int variant)
{
    if (!b) return fail(NLSE_E_INVAL, "NULL batch");
    if (variant < 0 || variant > 1) return fail(NLSE_E_INVAL, "variant out of range");
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
        b->lds = batch_lds_for(b->prec, b->variant, b->max1d, b->has2d);
        HIPTRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
        hipError_t e = launch_batch(b->prec, b->variant, b->d_items, b->d_order, (int)b->ctx.size(), b->d_queue,
                                    nsteps, b->grid, b->lds, b->cap);
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

// Autotuner of the batched launch: times `nsteps` steps of every variant and keeps the
// fastest.  The masters Psi^n of all instances are saved before and restored after
// each trial (device-to-device), so the integration state is unchanged.
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
    for (int v = 0; v < 2 && he == hipSuccess && !rc; ++v) {
        b->variant = v;
        he = hipEventRecord(e0, b->stream);
        if (he == hipSuccess) rc = nlse_batch_step(b, nsteps);
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
