// Auxiliary kernels: boundary-face closure values, field conversion, and the
// deterministic FP64 reductions (mass, energy, extrema of s|Psi|^2 - V).
#include "kernels.h"
#include "point.h"

namespace nlse {

// ----------------------------------------------------------------- helpers --

template <typename M>
__device__ __forceinline__ double abs2d(const C<M> &u) { return (double)u.x * u.x + (double)u.y * u.y; }

__device__ __forceinline__ bool on_boundary(const Layout &L, int64_t x, int64_t y, int64_t z)
{
    if (x == 0 || x == L.nx) return true;
    if (L.dim > 1 && (y == 0 || y == L.ny)) return true;
    if (L.dim > 2 && (z == 0 || z == L.nz)) return true;
    return false;
}

// ------------------------------------------------- boundary-face closure ----
//
// For a face node q normal to axis a (boundary in axis a only):
//   D^a_q = Lap_b(q) - sum_{b != a} delta_b^2 Psi_q,   Lap_b = -(s|Psi_q|^2 - V_q) Psi_q / a
// (Eq. dbc_lap).  Computed in the master precision, stored in the stage precision.
// Arrays per axis a: [2][nodes of the face], side 0 = index 0, side 1 = index n_a.
//   a = x: face index (z, y) -> z*(ny+1) + y
//   a = y: face index (z, x) -> z*(nx+1) + x
//   a = z: face index (y, x) -> y*(nx+1) + x
template <typename R, typename M>
__global__ void boundary_d_kernel(const C<M> *psi, const R *V, Layout L, Coeffs c, C<R> *DBx,
                                  C<R> *DBy, C<R> *DBz)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int axis = blockIdx.y, side = blockIdx.z;
    const int64_t nn[3] = {L.nx, L.ny, L.nz};
    if (axis >= L.dim) return;
    // the two tangential axes (unused ones have 0 intervals)
    const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
    const int64_t m1 = nn[t1] + 1, m2 = t2 < L.dim ? nn[t2] + 1 : 1;
    if (i >= m1 * m2) return;
    int64_t co[3] = {0, 0, 0};
    co[axis] = side ? nn[axis] : 0;
    co[t1] = i % m1;
    if (t2 < L.dim) co[t2] = i / m1;
    const M ih2 = (M)c.ih2;
    const int64_t p = L.idx(co[0], co[1], co[2]);
    const C<M> u = psi[p];
    const M Vq = V ? (M)V[p] : M(0);
    C<M> acc = dirichlet_lapb<M>(u, Vq, (M)c.s, (M)c.ia);
    const int tang[2] = {t1, t2};
    for (int k = 0; k < 2; ++k) {
        const int b = tang[k];
        if (b >= L.dim) continue;
        if (co[b] == 0 || co[b] == nn[b]) continue;   // edge/corner node: never read
        int64_t cp[3] = {co[0], co[1], co[2]}, cm[3] = {co[0], co[1], co[2]};
        cp[b] += 1;
        cm[b] -= 1;
        const C<M> up = psi[L.idx(cp[0], cp[1], cp[2])], um = psi[L.idx(cm[0], cm[1], cm[2])];
        acc = csub<M>(acc, d2<M>(um, u, up, ih2));
    }
    C<R> *dst = axis == 0 ? DBx : axis == 1 ? DBy : DBz;
    dst[side * m1 * m2 + i] = cvt<R, M>(acc);
}

template <typename R, typename M>
static hipError_t launch_bd(const void *psin, const void *V, const Layout &L, const Coeffs &c,
                            void *DB[3], hipStream_t st)
{
    const int64_t nn[3] = {L.nx, L.ny, L.nz};
    int64_t maxf = 1;
    for (int a = 0; a < L.dim; ++a) {
        int64_t f = 1;
        for (int b = 0; b < L.dim; ++b)
            if (b != a) f *= nn[b] + 1;
        if (f > maxf) maxf = f;
    }
    dim3 grid((unsigned)((maxf + 255) / 256), (unsigned)L.dim, 2);
    hipLaunchKernelGGL((boundary_d_kernel<R, M>), grid, dim3(256), 0, st, (const C<M> *)psin,
                       (const R *)V, L, c, (C<R> *)DB[0], (C<R> *)DB[1], (C<R> *)DB[2]);
    return hipGetLastError();
}

hipError_t launch_boundary_d(Prec prec, const void *psin, const void *V, const Layout &L,
                             const Coeffs &c, void *DB[3], hipStream_t st)
{
    // V is stored in the stage precision (double for F64, float for F32 / MIXED)
    switch (prec) {
    case P_F64: return launch_bd<double, double>(psin, V, L, c, DB, st);
    case P_F32: return launch_bd<float, float>(psin, V, L, c, DB, st);
    default: return launch_bd<float, double>(psin, V, L, c, DB, st);
    }
}

// ------------------------------------------------- 1D boundary closure ----
//
// For both ends b of a 1D field (node 0, node n) the step-1 boundary value D_b from the master
// field in FP64 -- Eq. dbc_lap (Dirichlet) or Eq. msdbc_lap (MSD: D_b = [Re(D_{b-1}/Psi_{b-1})
// + (N_{b-1} - N_b)/a] Psi_b with N = s|Psi|^2 - V, the ratio dropped when Psi_{b-1} = 0) -- into
// DB[side] (stage precision), and under MSD the step-size bound's boundary term
// max over the ends of (h^2/a) |F_{b-1} / Psi_{b-1}| into *bound_out, with F_{b-1} the
// right-hand side at b-1 from the 2SHOC combination that uses D_b.  One thread per end.
template <typename R, typename M>
__global__ void edges1d_kernel(const C<M> *psi, const R *V, Layout L, Coeffs c, int msd, double h2a, C<R> *DB,
                               double *bound_out)
{
    __shared__ double term[2];
    const int side = threadIdx.x;
    if (side < 2) {
        const int64_t n = L.nx;
        auto node = [&](int k) { return side ? n - k : (int64_t)k; };   // k-th node inward from the end
        auto u = [&](int k) {
            const C<M> v = psi[L.ox + node(k)];
            return make_double2((double)v.x, (double)v.y);
        };
        auto Vq = [&](int k) { return V ? (double)V[L.ox + node(k)] : 0.0; };
        auto N = [&](int k) {
            const double2 w = u(k);
            return c.s * (w.x * w.x + w.y * w.y) - Vq(k);
        };
        const double2 ub = u(0);
        double2 db;
        double t = 0.0;
        if (!msd) {
            const double f = -N(0) / c.a;
            db = make_double2(f * ub.x, f * ub.y);
        } else {
            auto d2 = [&](int k) {   // second difference at node k inward (neighbours k-1, k+1)
                const double2 lo = u(k - 1), m = u(k), hi = u(k + 1);
                return make_double2(c.ih2 * ((lo.x - 2.0 * m.x) + hi.x), c.ih2 * ((lo.y - 2.0 * m.y) + hi.y));
            };
            const double2 u1 = u(1), D1 = d2(1), D2 = d2(2);
            const double den = u1.x * u1.x + u1.y * u1.y;
            const double ratio = den != 0.0 ? (D1.x * u1.x + D1.y * u1.y) / den : 0.0;
            const double f = ratio + (N(1) - N(0)) / c.a;
            db = make_double2(f * ub.x, f * ub.y);
            const double lx = c.c76 * D1.x - (D2.x + db.x) * c.c112, ly = c.c76 * D1.y - (D2.y + db.y) * c.c112;
            const double zx = c.a * lx + N(1) * u1.x, zy = c.a * ly + N(1) * u1.y;   // F_{b-1} = i z
            if (den != 0.0) t = h2a * sqrt((zx * zx + zy * zy) / den);
        }
        DB[side] = cvt<R, double>(db);
        term[side] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0 && bound_out) *bound_out = fmax(term[0], term[1]);
}

hipError_t launch_edges1d(Prec prec, const void *psin, const void *V, const Layout &L, const Coeffs &c, bool msd,
                          double h2a, void *DB, double *bound_out, hipStream_t st)
{
    switch (prec) {
    case P_F64:
        hipLaunchKernelGGL((edges1d_kernel<double, double>), dim3(1), dim3(64), 0, st, (const C<double> *)psin,
                           (const double *)V, L, c, (int)msd, h2a, (C<double> *)DB, bound_out);
        break;
    case P_F32:
        hipLaunchKernelGGL((edges1d_kernel<float, float>), dim3(1), dim3(64), 0, st, (const C<float> *)psin,
                           (const float *)V, L, c, (int)msd, h2a, (C<float> *)DB, bound_out);
        break;
    default:
        hipLaunchKernelGGL((edges1d_kernel<float, double>), dim3(1), dim3(64), 0, st, (const C<double> *)psin,
                           (const float *)V, L, c, (int)msd, h2a, (C<float> *)DB, bound_out);
    }
    return hipGetLastError();
}

// ------------------------------------------------------ master -> stage ----

template <typename R, typename M>
__global__ void m2s_kernel(const C<M> *src, C<R> *dst, int64_t total)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = cvt<R, M>(src[i]);
}

hipError_t launch_master_to_stage(Prec prec, const void *psin, void *dst, const Layout &L, hipStream_t st)
{
    const unsigned blocks = (unsigned)((L.total + 255) / 256 < 65536 ? (L.total + 255) / 256 : 65536);
    switch (prec) {
    case P_F64:
        hipLaunchKernelGGL((m2s_kernel<double, double>), dim3(blocks), dim3(256), 0, st,
                           (const C<double> *)psin, (C<double> *)dst, L.total);
        break;
    case P_F32:
        hipLaunchKernelGGL((m2s_kernel<float, float>), dim3(blocks), dim3(256), 0, st,
                           (const C<float> *)psin, (C<float> *)dst, L.total);
        break;
    default:
        hipLaunchKernelGGL((m2s_kernel<float, double>), dim3(blocks), dim3(256), 0, st,
                           (const C<double> *)psin, (C<float> *)dst, L.total);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------- reductions --
//
// Pass 1: block b sums rows b, b + G, b + 2G, ... (a row = the nx + 1 nodes of one
// (y, z)); each thread accumulates its strided nodes in order, then a fixed
// shared-memory tree.  Pass 2: one block sums the G partials the same way.  The
// order depends only on the layout, so results are reproducible bit for bit.

constexpr int RED_BLOCKS = 1024, RED_THREADS = 256;
int reduce_partials() { return RED_BLOCKS; }

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ void finish_sum_kernel(const double *partials, int np, double scale, double *out)
{
    __shared__ double sh[RED_THREADS];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += RED_THREADS) acc += partials[i];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) out[0] = r * scale;
}

template <typename M>
__global__ __launch_bounds__(RED_THREADS) void mass_kernel(const C<M> *psi, Layout L, double *partials)
{
    __shared__ double sh[RED_THREADS];
    const int64_t rows = L.py * (L.nz + 1);
    double acc = 0.0;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int64_t y = row % L.py, z = row / L.py;
        for (int64_t x = threadIdx.x; x <= L.nx; x += RED_THREADS) acc += abs2d<M>(psi[L.idx(x, y, z)]);
    }
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

hipError_t launch_mass(Prec prec, const void *psin, const Layout &L, double *partials,
                       double *dev_out, hipStream_t st, double scale)
{
    if (prec == P_F32)
        hipLaunchKernelGGL((mass_kernel<float>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const C<float> *)psin, L, partials);
    else
        hipLaunchKernelGGL((mass_kernel<double>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const C<double> *)psin, L, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(RED_THREADS), 0, st, partials, RED_BLOCKS, scale,
                       dev_out);
    return hipGetLastError();
}

// Energy density at an interior node, in FP64 from the stored field, with the
// per-axis 2SHOC Laplacian and the boundary-face closure values DB.
template <typename M, typename R>
__device__ double energy_at(const C<M> *psi, const R *V, const C<R> *const *DB, const Layout &L,
                            const Coeffs &c, int64_t x, int64_t y, int64_t z)
{
    const int64_t co[3] = {x, y, z};
    const int64_t nn[3] = {L.nx, L.ny, L.nz};
    const double ih2 = c.ih2;
    auto val = [&](int64_t a0, int64_t a1, int64_t a2) {
        const C<M> v = psi[L.idx(a0, a1, a2)];
        return make_double2((double)v.x, (double)v.y);
    };
    const double2 u = val(x, y, z);
    double lx = 0.0, ly = 0.0;
    for (int a = 0; a < L.dim; ++a) {
        // D^a at offsets -1, 0, +1 along a
        double2 d[3];
        for (int o = -1; o <= 1; ++o) {
            int64_t q[3] = {co[0], co[1], co[2]};
            q[a] += o;
            if (q[a] == 0 || q[a] == nn[a]) {
                int64_t fi;
                if (a == 0) fi = q[2] * (L.ny + 1) + q[1];
                else if (a == 1) fi = q[2] * (L.nx + 1) + q[0];
                else fi = q[1] * (L.nx + 1) + q[0];
                int64_t fsz = 1;
                for (int b = 0; b < L.dim; ++b)
                    if (b != a) fsz *= nn[b] + 1;
                const C<R> db = DB[a][(q[a] ? fsz : 0) + fi];
                d[o + 1] = make_double2((double)db.x, (double)db.y);
            } else {
                int64_t qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
                qp[a] += 1;
                qm[a] -= 1;
                const double2 c0 = val(q[0], q[1], q[2]), cp = val(qp[0], qp[1], qp[2]),
                              cm = val(qm[0], qm[1], qm[2]);
                d[o + 1] = make_double2(ih2 * ((cp.x - 2.0 * c0.x) + cm.x), ih2 * ((cp.y - 2.0 * c0.y) + cm.y));
            }
        }
        lx += c.c76 * d[1].x - c.c112 * (d[2].x + d[0].x);
        ly += c.c76 * d[1].y - c.c112 * (d[2].y + d[0].y);
    }
    const double r2 = u.x * u.x + u.y * u.y;
    const double Vq = V ? (double)V[L.idx(x, y, z)] : 0.0;
    return -c.a * (u.x * lx + u.y * ly) + Vq * r2 - 0.5 * c.s * r2 * r2;
}

template <typename M, typename R>
__global__ __launch_bounds__(RED_THREADS) void energy_kernel(const C<M> *psi, const R *V, const C<R> *DBx,
                                                            const C<R> *DBy, const C<R> *DBz, Layout L,
                                                            Coeffs c, double *partials)
{
    __shared__ double sh[RED_THREADS];
    const C<R> *DB[3] = {DBx, DBy, DBz};
    const int64_t rows = L.py * (L.nz + 1);
    double acc = 0.0;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int64_t y = row % L.py, z = row / L.py;
        if ((L.dim > 1 && (y == 0 || y == L.ny)) || (L.dim > 2 && (z == 0 || z == L.nz))) continue;
        for (int64_t x = 1 + threadIdx.x; x < L.nx; x += RED_THREADS)
            acc += energy_at<M, R>(psi, V, DB, L, c, x, y, z);
    }
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

hipError_t launch_energy(Prec prec, const void *psin, const void *V, const void *const DB[3],
                         const Layout &L, const Coeffs &c, double *partials, double *dev_out,
                         hipStream_t st)
{
    switch (prec) {
    case P_F64:
        hipLaunchKernelGGL((energy_kernel<double, double>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const C<double> *)psin, (const double *)V, (const C<double> *)DB[0],
                           (const C<double> *)DB[1], (const C<double> *)DB[2], L, c, partials);
        break;
    case P_F32:
        hipLaunchKernelGGL((energy_kernel<float, float>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const C<float> *)psin, (const float *)V, (const C<float> *)DB[0],
                           (const C<float> *)DB[1], (const C<float> *)DB[2], L, c, partials);
        break;
    default:
        hipLaunchKernelGGL((energy_kernel<double, float>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const C<double> *)psin, (const float *)V, (const C<float> *)DB[0],
                           (const C<float> *)DB[1], (const C<float> *)DB[2], L, c, partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double scale = 1.0;
    const double h = 1.0 / sqrt(c.ih2);
    for (int a = 0; a < L.dim; ++a) scale *= h;
    hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(RED_THREADS), 0, st, partials, RED_BLOCKS, scale,
                       dev_out);
    return hipGetLastError();
}

template <typename M, typename R>
__global__ __launch_bounds__(RED_THREADS) void minmax_kernel(const C<M> *psi, const R *V, Layout L, double s,
                                                            double *partials)
{
    __shared__ double shmin[RED_THREADS], shmax[RED_THREADS];
    const int64_t rows = L.py * (L.nz + 1);
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int64_t y = row % L.py, z = row / L.py;
        if ((L.dim > 1 && (y == 0 || y == L.ny)) || (L.dim > 2 && (z == 0 || z == L.nz))) continue;
        for (int64_t x = 1 + threadIdx.x; x < L.nx; x += RED_THREADS) {
            const int64_t p = L.idx(x, y, z);
            const double v = s * abs2d<M>(psi[p]) - (V ? (double)V[p] : 0.0);
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
    }
    shmin[threadIdx.x] = lo;
    shmax[threadIdx.x] = hi;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            shmin[threadIdx.x] = fmin(shmin[threadIdx.x], shmin[threadIdx.x + w]);
            shmax[threadIdx.x] = fmax(shmax[threadIdx.x], shmax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = shmin[0];
        partials[2 * blockIdx.x + 1] = shmax[0];
    }
}

__global__ void finish_minmax_kernel(const double *partials, int np, double *out)
{
    __shared__ double shmin[RED_THREADS], shmax[RED_THREADS];
    double lo = INFINITY, hi = -INFINITY;
    for (int i = threadIdx.x; i < np; i += RED_THREADS) {
        lo = fmin(lo, partials[2 * i]);
        hi = fmax(hi, partials[2 * i + 1]);
    }
    shmin[threadIdx.x] = lo;
    shmax[threadIdx.x] = hi;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            shmin[threadIdx.x] = fmin(shmin[threadIdx.x], shmin[threadIdx.x + w]);
            shmax[threadIdx.x] = fmax(shmax[threadIdx.x], shmax[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = shmin[0];
        out[1] = shmax[0];
    }
}

hipError_t launch_minmax_nonlin(Prec prec, const void *psin, const void *V, const Layout &L, double s,
                                double *partials, double *dev_out, hipStream_t st)
{
    if (prec == P_F32)
        hipLaunchKernelGGL((minmax_kernel<float, float>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const C<float> *)psin, (const float *)V, L, s, partials);
    else if (prec == P_F64)
        hipLaunchKernelGGL((minmax_kernel<double, double>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const C<double> *)psin, (const double *)V, L, s, partials);
    else
        hipLaunchKernelGGL((minmax_kernel<double, float>), dim3(RED_BLOCKS), dim3(RED_THREADS), 0, st,
                           (const C<double> *)psin, (const float *)V, L, s, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finish_minmax_kernel, dim3(1), dim3(RED_THREADS), 0, st, partials, RED_BLOCKS, dev_out);
    return hipGetLastError();
}

}  // namespace nlse
