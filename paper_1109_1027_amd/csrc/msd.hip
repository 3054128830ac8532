// The modulus-squared Dirichlet (MSD) boundary in 2D and 3D (Sec. 3.2).
//
// The paper gives the MSD rule for a boundary node b in terms of b-1, the nearest
// interior node in the normal direction, and notes that it carries over to
// several dimensions.  Here b-1 is the closest interior node: one step inward
// along every axis on which b is a boundary node (the normal neighbour on a face,
// the diagonal interior neighbour on an edge or corner, where no normal exists).
//
//   step 1 (Eq. msdbc_lap):  Lap_b = [Re(D_{b-1} / Psi_{b-1}) + (N_{b-1} - N_b) / a] Psi_b
//   time derivative (Eq. msdbc_ut):  F_b = i Im(F_{b-1} / Psi_{b-1}) Psi_b
//   N = s |Psi|^2 - V (Eq. nbnb1); a zero Psi_{b-1} drops the ratio term.
//
// The interior stage kernels (per-axis 2SHOC) read, on a face node normal to axis
// a, the value D^a_b = Lap_b - (second differences along the face), the closure
// under which the per-axis form equals the single-storage one.  Under Dirichlet
// those values are constants; under MSD they follow the field, so every RK4 stage
// runs two launches:
//   1. msd_stage_kernel   one thread per boundary node: D^a_b on the face nodes from
//      the stage's input field, for the interior launch; and F_b from F_{b-1}
//      (interior first, boundary second), with F_{b-1} recomputed from the same input
//      and face values formed on the spot, then the stage's RK4 array operations on
//      the boundary node.  Neither part reads what the interior launch writes.
//   2. the interior stage kernel (unchanged: it reads the face values).
// The boundary work is O(n^(d-1)) against the interior's O(n^d).  msd_face_kernel
// alone serves the bound and the energy.
#include "kernels.h"
#include "point.h"

namespace nlse {

namespace {

template <typename T, typename U> struct same_m { static constexpr bool v = false; };
template <typename T> struct same_m<T, T> { static constexpr bool v = true; };

// A node (x, y, z); the axis is selected by value, never by a dynamic array index,
// so nothing lands in scratch memory.
struct Node {
    int x, y, z;
    __device__ __forceinline__ int at(int a) const { return a == 0 ? x : a == 1 ? y : z; }
    __device__ __forceinline__ void set(int a, int v)
    {
        if (a == 0) x = v;
        else if (a == 1) y = v;
        else z = v;
    }
};

__device__ __forceinline__ int ext(const Layout &L, int a) { return (int)(a == 0 ? L.nx : a == 1 ? L.ny : L.nz); }

__device__ __forceinline__ bool on_bnd(const Layout &L, const Node &q, int a)
{
    return a < L.dim && (q.at(a) == 0 || q.at(a) == ext(L, a));
}

__device__ __forceinline__ Node step(Node q, int a, int d)
{
    q.set(a, q.at(a) + d);
    return q;
}

// Index of node q within the face normal to axis a (layout of the face arrays):
// a = x: z (ny+1) + y;  a = y: z (nx+1) + x;  a = z: y (nx+1) + x.
__device__ __forceinline__ int64_t face_index(const Layout &L, int a, const Node &q)
{
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    int64_t fi = q.at(t1);
    if (t2 < L.dim) fi += (int64_t)q.at(t2) * (ext(L, t1) + 1);
    return fi;
}

__device__ __forceinline__ int64_t face_size(const Layout &L, int a)
{
    int64_t f = 1;
    for (int b = 0; b < L.dim; ++b)
        if (b != a) f *= ext(L, b) + 1;
    return f;
}

// The boundary node of face (axis a, side) with face index fi.
__device__ __forceinline__ Node face_node(const Layout &L, int a, int side, int64_t fi)
{
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    Node q{0, 0, 0};
    q.set(a, side ? ext(L, a) : 0);
    const int64_t m1 = ext(L, t1) + 1;
    q.set(t1, (int)(fi % m1));
    if (t2 < L.dim) q.set(t2, (int)(fi / m1));
    return q;
}

// b-1 of the MSD rule: one step inward along every boundary axis of b.
__device__ __forceinline__ Node inner(const Layout &L, Node b)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a >= L.dim) break;
        if (b.at(a) == 0) b.set(a, 1);
        else if (b.at(a) == ext(L, a)) b.set(a, ext(L, a) - 1);
    }
    return b;
}

template <typename IN, typename R>
struct Field {
    const C<IN> *in;
    const R *V;
    Layout L;
    __device__ __forceinline__ C<R> psi(const Node &q) const { return cvt<R, IN>(in[L.idx(q.x, q.y, q.z)]); }
    __device__ __forceinline__ R pot(const Node &q) const { return V ? V[L.idx(q.x, q.y, q.z)] : R(0); }
    // delta_a^2 Psi at q (q +- e_a inside the grid)
    __device__ __forceinline__ C<R> d2a(const Node &q, int a, R ih2) const
    {
        return d2<R>(psi(step(q, a, -1)), psi(q), psi(step(q, a, 1)), ih2);
    }
    // h^2 delta_a^2 Psi at q, unscaled (as the interior kernels form it)
    __device__ __forceinline__ C<R> d2u_a(const Node &q, int a) const
    {
        return d2u<R>(psi(step(q, a, -1)), psi(q), psi(step(q, a, 1)));
    }
};

// The face value D^a_b at the face node b (normal to a, on no other face): the MSD step-1
// value of Eq. msdbc_lap, from the full step-1 value at b-1, minus the second differences
// along the face.
template <typename IN, typename R, int DIM>
__device__ __forceinline__ C<R> face_closure(const Field<IN, R> &f, const Coeffs &cf, int a, const Node &b)
{
#pragma clang fp contract(off)
    const int side = b.at(a) == 0 ? 0 : 1;
    const R ih2 = (R)cf.ih2, s = (R)cf.s;
    const Node q = step(b, a, side ? -1 : 1);
    const C<R> ub = f.psi(b), uq = f.psi(q);
    C<R> Dq = czero<R>();   // the full step-1 value at b-1 (Eqs. 2d2shocs1, 3d2shocs)
#pragma unroll
    for (int t = 0; t < DIM; ++t) Dq = cadd<R>(Dq, f.d2a(q, t, ih2));
    const R ratio = re_div<R>(Dq, uq);
    const R fac = ratio + (nonlin<R>(uq, f.pot(q), s) - nonlin<R>(ub, f.pot(b), s)) * (R)cf.ia;
    C<R> Db = mk<R>(fac * ub.x, fac * ub.y);   // Lap_b
#pragma unroll
    for (int t = 0; t < DIM; ++t)
        if (t != a) Db = csub<R>(Db, f.d2a(b, t, ih2));
    return Db;
}

// Face values as the interior kernels read them: from the face arrays ...
template <typename R>
struct StoredFaces {
    const C<R> *DB[3];
    Layout L;
    __device__ __forceinline__ C<R> operator()(int a, const Node &r) const
    {
        const int side = r.at(a) == 0 ? 0 : 1;
        return DB[a][side * face_size(L, a) + face_index(L, a, r)];
    }
};

// ... or formed from the field on the spot (while another thread may be writing the arrays).
template <typename IN, typename R, int DIM>
struct DirectFaces {
    Field<IN, R> f;
    Coeffs cf;
    __device__ __forceinline__ C<R> operator()(int a, const Node &r) const { return face_closure<IN, R, DIM>(f, cf, a, r); }
};

// ... or, for the thread that has just formed the value at its own face node b, that value
// there and formed on the spot elsewhere.
template <typename IN, typename R, int DIM>
struct KnownFace {
    DirectFaces<IN, R, DIM> direct;
    int a;
    Node b;
    C<R> value;
    bool known;
    __device__ __forceinline__ C<R> operator()(int ax, const Node &r) const
    {
        if (known && ax == a && r.x == b.x && r.y == b.y && r.z == b.z) return value;
        return direct(ax, r);
    }
};

// F at the interior node q, per-axis 2SHOC (Eqs. 2d2shocMs1-2, 3d2shocMs1-2) with the face
// values where q's neighbour along an axis is a boundary node.  Formed exactly as the interior
// stage kernels form it (unscaled second differences, face values times h^2, a and 1/h^2 folded
// into the step-2 coefficients), so F_{b-1} of the boundary rule is bitwise the interior
// kernels' F at b-1.
template <typename IN, typename R, int DIM, typename Faces>
__device__ C<R> interior_F(const Field<IN, R> &f, const Faces &face_value, const Coeffs &cf, const Node &q)
{
    const Step2Coef<R> lc = step2_coef<R>(cf.a, cf.c76, cf.c112, cf.ih2);
    C<R> dc[3], dl[3], dr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dc[a] = dl[a] = dr[a] = czero<R>();
        if (a >= DIM) continue;
        dc[a] = f.d2u_a(q, a);
        const Node lo = step(q, a, -1), hi = step(q, a, 1);
        dl[a] = lo.at(a) == 0 ? unscaled<R>(face_value(a, lo), lc.h2) : f.d2u_a(lo, a);
        dr[a] = hi.at(a) == ext(f.L, a) ? unscaled<R>(face_value(a, hi), lc.h2) : f.d2u_a(hi, a);
    }
    C<R> alap;
    if constexpr (DIM == 2) {
        alap = lap2a<R>(dc[0], dc[1], dl[0], dr[0], dl[1], dr[1], lc.A76, lc.A112);
    } else {
        alap = lap3<R>(dc[0], dc[1], dc[2], dl[0], dr[0], dl[1], dr[1], dl[2], dr[2], lc.A76, lc.A112);
    }
    return rhs_a<R>(alap, f.psi(q), f.pot(q), (R)cf.s);
}

// Im(F_q / Psi_q), 0 when Psi_q = 0.
template <typename R>
__device__ __forceinline__ R phase_rate(const C<R> &F, const C<R> &u)
{
    return im_div<R>(F, u);
}

// ---- 1. face values D^a_b from the stage input -------------------------------------------

template <typename IN, typename R, int DIM>
__global__ void msd_face_kernel(Field<IN, R> f, Coeffs cf, C<R> *DBx, C<R> *DBy, C<R> *DBz)
{
    const int a = blockIdx.y, side = blockIdx.z;
    const Layout &L = f.L;
    if (a >= L.dim) return;
    const int64_t fi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (fi >= face_size(L, a)) return;
    const Node b = face_node(L, a, side, fi);
#pragma unroll
    for (int t = 0; t < 3; ++t)
        if (t != a && on_bnd(L, b, t)) return;   // edge / corner: never read by the stage kernels
    C<R> *dst = a == 0 ? DBx : a == 1 ? DBy : DBz;
    dst[side * face_size(L, a) + fi] = face_closure<IN, R, DIM>(f, cf, a, b);
}

template <typename IN, typename R>
static hipError_t launch_faces(const void *in, const void *V, const Layout &L, const Coeffs &c, void *const DB[3],
                               hipStream_t st)
{
    int64_t maxf = 1;
    for (int a = 0; a < L.dim; ++a) {
        int64_t f = 1;
        for (int b = 0; b < L.dim; ++b)
            if (b != a) f *= (b == 0 ? L.nx : b == 1 ? L.ny : L.nz) + 1;
        if (f > maxf) maxf = f;
    }
    Field<IN, R> f{(const C<IN> *)in, (const R *)V, L};
    dim3 grid((unsigned)((maxf + 255) / 256), (unsigned)L.dim, 2);
    if (L.dim == 3)
        hipLaunchKernelGGL((msd_face_kernel<IN, R, 3>), grid, dim3(256), 0, st, f, c, (C<R> *)DB[0], (C<R> *)DB[1],
                           (C<R> *)DB[2]);
    else
        hipLaunchKernelGGL((msd_face_kernel<IN, R, 2>), grid, dim3(256), 0, st, f, c, (C<R> *)DB[0], (C<R> *)DB[1],
                           (C<R> *)DB[2]);
    return hipGetLastError();
}

// ---- 3. boundary F_b and the stage's RK4 operations on the boundary --------------------------

// Every boundary node once: the face of the lowest axis on which it lies.
__device__ __forceinline__ bool owner(const Layout &L, const Node &b, int a)
{
#pragma unroll
    for (int t = 0; t < 3; ++t)
        if (t < a && on_bnd(L, b, t)) return false;
    return true;
}

// Every load of a thread is issued before its first store: a store in between would make
// the compiler keep the loads behind it (the arrays may alias, as far as it knows) and so
// add a memory round trip per group of loads to a launch that is all latency.
template <typename IN, typename R, typename M, int DIM>
__global__ __launch_bounds__(256) void msd_stage_kernel(Field<IN, R> f, StageArgs A, C<R> *DBx, C<R> *DBy, C<R> *DBz)
{
    const int a = blockIdx.y, side = blockIdx.z;
    const Layout &L = f.L;
    if (a >= DIM) return;
    // consecutive face rows on one XCD, whose L2 then holds the rows that neighbours share
    const int64_t fi = xcd_remap(blockIdx.x, gridDim.x) * (int64_t)blockDim.x + threadIdx.x;
    if (fi >= face_size(L, a)) return;
    const Node b = face_node(L, a, side, fi);
    bool face = true;   // on no other face: the interior launch reads its D^a_b
#pragma unroll
    for (int t = 0; t < DIM; ++t)
        if (t != a && on_bnd(L, b, t)) face = false;
    const bool own = owner(L, b, a);
    const int64_t p = L.idx(b.x, b.y, b.z);
    C<M> *psin = (C<M> *)A.psin;
    C<R> *K = (C<R> *)A.K;
    C<R> *out = (C<R> *)A.out;
    C<M> pn = mk<M>(M(0), M(0));
    C<R> kt = czero<R>();
    if (own && (A.stage >= 2 || !same_m<IN, R>::v)) pn = psin[p];
    if (own && A.stage >= 2) kt = K[p];
    const DirectFaces<IN, R, DIM> direct{f, A.c};
    KnownFace<IN, R, DIM> faces{direct, a, b, czero<R>(), false};
    if (face) {
        faces.value = direct(a, b);
        faces.known = true;
    }
    C<R> F = czero<R>(), ub = czero<R>();
    if (own) {
        const Node q = inner(L, b);
        const C<R> uq = f.psi(q);
        ub = f.psi(b);
        F = msd_fb<R>(phase_rate<R>(interior_F<IN, R, DIM>(f, faces, A.c, q), uq), ub);
    }
    if (face) {
        C<R> *dst = a == 0 ? DBx : a == 1 ? DBy : DBz;
        dst[side * face_size(L, a) + fi] = faces.value;
    }
    if (!own) return;
    const R ck = (R)A.c.ck;
    if (A.stage == 1) {
        const C<M> base = same_m<IN, R>::v ? cvt<M, R>(ub) : pn;
        K[p] = F;
        out[p] = cvt<R, M>(axpy_m<R, M>(base, ck, F));
    } else if (A.stage <= 3) {
        K[p] = kacc<R>(kt, F);
        out[p] = cvt<R, M>(axpy_m<R, M>(pn, ck, F));
    } else {
        psin[p] = axpy_m<R, M>(pn, ck, cadd<R>(kt, F));
    }
}

template <typename IN, typename R, typename M>
static hipError_t launch_stage_bnd(const StageArgs &A, void *const DB[3], hipStream_t st)
{
    const Layout &L = A.L;
    int64_t maxf = 1;
    for (int a = 0; a < L.dim; ++a) {
        int64_t f = 1;
        for (int b = 0; b < L.dim; ++b)
            if (b != a) f *= (b == 0 ? L.nx : b == 1 ? L.ny : L.nz) + 1;
        if (f > maxf) maxf = f;
    }
    Field<IN, R> f{(const C<IN> *)A.in, (const R *)A.V, L};
    // a 2D boundary has a few thousand nodes and the launch is latency: one-wave blocks spread
    // them over four times as many CUs
    const int bs = L.dim == 3 ? 256 : 64;
    dim3 grid((unsigned)((maxf + bs - 1) / bs), (unsigned)L.dim, 2);
    if (L.dim == 3)
        hipLaunchKernelGGL((msd_stage_kernel<IN, R, M, 3>), grid, dim3(bs), 0, st, f, A, (C<R> *)DB[0],
                           (C<R> *)DB[1], (C<R> *)DB[2]);
    else
        hipLaunchKernelGGL((msd_stage_kernel<IN, R, M, 2>), grid, dim3(bs), 0, st, f, A, (C<R> *)DB[0],
                           (C<R> *)DB[1], (C<R> *)DB[2]);
    return hipGetLastError();
}

// ---- the bound's boundary term: max over b-1 of (h^2/a) |F_{b-1} / Psi_{b-1}| -----------------

template <typename IN, typename R, int DIM>
__global__ void msd_bound_kernel(Field<IN, R> f, Coeffs cf, const void *DB0, const void *DB1, const void *DB2,
                                 double h2a, unsigned long long *out)
{
    const int a = blockIdx.y, side = blockIdx.z;
    const Layout &L = f.L;
    if (a >= L.dim) return;
    const int64_t fi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (fi >= face_size(L, a)) return;
    const Node b = face_node(L, a, side, fi);
    if (!owner(L, b, a)) return;
    const StoredFaces<R> faces{{(const C<R> *)DB0, (const C<R> *)DB1, (const C<R> *)DB2}, L};
    const Node q = inner(L, b);
    const C<R> uq = f.psi(q);
    const double den = (double)uq.x * uq.x + (double)uq.y * uq.y;
    if (den == 0.0) return;
    const C<R> F = interior_F<IN, R, DIM>(f, faces, cf, q);
    const double B = h2a * sqrt(((double)F.x * F.x + (double)F.y * F.y) / den);
    // non-negative doubles order as their bit patterns: the maximum is exact and order-free
    atomicMax(out, (unsigned long long)__double_as_longlong(B));
}

}  // namespace

hipError_t launch_msd_faces(Prec prec, bool master, const void *in, const void *V, const Layout &L,
                            const Coeffs &c, void *const DB[3], hipStream_t st)
{
    switch (prec) {
    case P_F64: return launch_faces<double, double>(in, V, L, c, DB, st);
    case P_F32: return launch_faces<float, float>(in, V, L, c, DB, st);
    default: return master ? launch_faces<double, float>(in, V, L, c, DB, st) : launch_faces<float, float>(in, V, L, c, DB, st);
    }
}

hipError_t launch_msd_stage(Prec prec, const StageArgs &a, void *const DB[3], hipStream_t st)
{
    switch (prec) {
    case P_F64: return launch_stage_bnd<double, double, double>(a, DB, st);
    case P_F32: return launch_stage_bnd<float, float, float>(a, DB, st);
    default:
        if (a.stage == 1) return launch_stage_bnd<double, float, double>(a, DB, st);
        return launch_stage_bnd<float, float, double>(a, DB, st);
    }
}

hipError_t launch_msd_bound(Prec prec, const void *psin, const void *V, const void *const DB[3], const Layout &L,
                            const Coeffs &c, double h2a, double *dev_out, hipStream_t st)
{
    hipError_t e = hipMemsetAsync(dev_out, 0, sizeof(double), st);
    if (e != hipSuccess) return e;
    int64_t maxf = 1;
    for (int a = 0; a < L.dim; ++a) {
        int64_t f = 1;
        for (int b = 0; b < L.dim; ++b)
            if (b != a) f *= (b == 0 ? L.nx : b == 1 ? L.ny : L.nz) + 1;
        if (f > maxf) maxf = f;
    }
    dim3 grid((unsigned)((maxf + 255) / 256), (unsigned)L.dim, 2);
    unsigned long long *o = (unsigned long long *)dev_out;
    switch (prec) {
    case P_F64:
        if (L.dim == 3)
            hipLaunchKernelGGL((msd_bound_kernel<double, double, 3>), grid, dim3(256), 0, st,
                               Field<double, double>{(const C<double> *)psin, (const double *)V, L}, c, DB[0], DB[1], DB[2],
                               h2a, o);
        else
            hipLaunchKernelGGL((msd_bound_kernel<double, double, 2>), grid, dim3(256), 0, st,
                               Field<double, double>{(const C<double> *)psin, (const double *)V, L}, c, DB[0], DB[1], DB[2],
                               h2a, o);
        break;
    case P_F32:
        if (L.dim == 3)
            hipLaunchKernelGGL((msd_bound_kernel<float, float, 3>), grid, dim3(256), 0, st,
                               Field<float, float>{(const C<float> *)psin, (const float *)V, L}, c, DB[0], DB[1], DB[2],
                               h2a, o);
        else
            hipLaunchKernelGGL((msd_bound_kernel<float, float, 2>), grid, dim3(256), 0, st,
                               Field<float, float>{(const C<float> *)psin, (const float *)V, L}, c, DB[0], DB[1], DB[2],
                               h2a, o);
        break;
    default:
        if (L.dim == 3)
            hipLaunchKernelGGL((msd_bound_kernel<double, float, 3>), grid, dim3(256), 0, st,
                               Field<double, float>{(const C<double> *)psin, (const float *)V, L}, c, DB[0], DB[1], DB[2],
                               h2a, o);
        else
            hipLaunchKernelGGL((msd_bound_kernel<double, float, 2>), grid, dim3(256), 0, st,
                               Field<double, float>{(const C<double> *)psin, (const float *)V, L}, c, DB[0], DB[1], DB[2],
                               h2a, o);
        break;
    }
    return hipGetLastError();
}

}  // namespace nlse
