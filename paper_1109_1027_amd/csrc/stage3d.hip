// Fused RK4-stage kernel for the 3D NLSE with the per-axis 2SHOC Laplacian
// (Sec. 2.3 Eqs. 3d2shocMs1-2, Sec. 3.1):
//   step 1   D^a = delta_a^2 Psi,  a in {x, y, z}
//   step 2   Lap = sum_a [ (7/6) D^a - (1/12)(D^a_{+a} + D^a_{-a}) ]
//   then F = i[a Lap + (s|Psi|^2 - V) Psi] and the stage's RK4 array operations.
//
// 2.5D scheme: a block owns a 64 x TYB column tile (x fastest, one coalesced row
// segment per wave) and marches along z through TZ planes.  Each thread keeps its
// column's Psi at z-2..z+2 and D^z at z-1..z+1 in registers; the current plane of
// Psi (with a 2-node halo in x and y) and the in-plane D^x, D^y (with a 1-node
// halo) go through LDS.  No D value is ever written to global memory.
//
// Software pipelining: everything plane z+1 needs from global memory (Psi at
// z+3, the plane's x/y halo, and the update operands Psi^n, K_tot, V) is loaded
// while plane z is computed, so a plane never waits a full memory round trip.
// Barriers only order LDS (they wait on LDS counters, not on loads in flight).
//
// The kernel is bound by instruction issue as much as by memory, so all
// addressing is 32-bit element offsets computed once per thread (fields of up to
// 2^31 elements; the launcher checks) and advanced by one plane stride per z
// step; every validity test that does not depend on z is hoisted out of the
// march, the z tests are block-uniform, and the RK4 stage is a template
// parameter so each stage loads only what it uses.
//
// Face closure values D^a_b (boundary-face nodes) come from the face arrays: the
// Dirichlet constants of launch_boundary_d, or under MSD the values msd.hip forms
// from the stage's input before each launch; see stage2d.hip for why the per-axis
// and single-storage forms then coincide.
//
// Alternative Laplacians for comparison (ST, from StageArgs::stencil): the
// non-compact fourth-order 13-point cross (Sec. 2.3: the 3D counterpart of
// Eq. 2dnonhoc), one five-point difference per axis with the ghosts
// 2 Psi_b - Psi_{b+-1} + h^2 D^a_b one node beyond a face (their second difference at b is
// the face value of Eq. dbc_lap), read from the same plane
// buffer (two-node halo) and column queue (z-2..z+2); and the second-order
// central difference D^x + D^y + D^z.  Neither needs the D halos in LDS.
#include "kernels.h"
#include "point.h"

namespace nlse {

template <typename T, typename U> struct same3_t { static constexpr bool v = false; };
template <typename T> struct same3_t<T, T> { static constexpr bool v = true; };

template <typename IN, typename R, typename M, int TYB, int TZ, int STAGE, int ST>
__global__ __launch_bounds__(64 * TYB) void stage3d_kernel(StageArgs A, int tiles_x, int tiles_y)
{
    constexpr int W = 64, NT = 64 * TYB;
    static_assert(NT >= 4 * W, "y-halo load needs at least 256 threads");
    __shared__ C<R> sp[TYB + 4][W + 4];
    __shared__ C<R> sdx[TYB][W + 2];
    __shared__ C<R> sdy[TYB + 2][W];

    const int t = threadIdx.x, tx = t & 63, ty = t >> 6;
    const int nx = (int)A.L.nx, ny = (int)A.L.ny, nz = (int)A.L.nz;
    const int px = (int)A.L.px, ox = (int)A.L.ox;
    const int plane = px * (int)A.L.py;
    const int lb = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % tiles_x, by = (lb / tiles_x) % tiles_y, bz = lb / (tiles_x * tiles_y);
    const int x0 = 1 + W * bx, y0 = 1 + TYB * by, z0 = 1 + TZ * bz;
    const int x = x0 + tx, y = y0 + ty;
    const bool col_ok = x <= nx && y <= ny;
    const bool upd_col = x < nx && y < ny;
    const bool xface = col_ok && x == nx, yface = col_ok && y == ny;
    const int cidx = y * px + x + ox;                    // own column, plane 0

    const R s = (R)A.c.s;
    const Step2Coef<R> lc = step2_coef<R>(A.c.a, A.c.c76, A.c.c112, A.c.ih2);   // 1/h^2 and a folded in
    const R ck = (R)A.c.ck;
    const C<IN> *in = (const C<IN> *)A.in;
    const C<R> *DBx = (const C<R> *)A.DB[0];
    const C<R> *DBy = (const C<R> *)A.DB[1];
    const C<R> *DBz = (const C<R> *)A.DB[2];
    const R *V = (const R *)A.V;
    C<M> *psin = (C<M> *)A.psin;
    C<R> *K = (C<R> *)A.K;
    C<R> *out = (C<R> *)A.out;
    constexpr bool in_is_r = same3_t<IN, R>::v;
    const int fx = (nz + 1) * (ny + 1), fy = (nz + 1) * (nx + 1), fz = (ny + 1) * (nx + 1);

    // halo roles, fixed for the whole march
    const bool hx_role = t < 4 * TYB;
    int hx_idx = 0, hx_pos_r = 0, hx_pos_c = 0;
    bool hx_ok = false;
    if (hx_role) {
        const int r = t >> 2, k = t & 3;
        const int hc = x0 + (k == 0 ? -2 : k == 1 ? -1 : k == 2 ? W : W + 1), hr = y0 + r;
        hx_ok = hc >= 0 && hc <= nx && hr <= ny;
        hx_idx = hr * px + hc + ox;
        hx_pos_r = r + 2;
        hx_pos_c = k == 0 ? 0 : k == 1 ? 1 : k == 2 ? W + 2 : W + 3;
    }
    const bool hy_role = t < 4 * W;
    int hy_idx = 0, hy_pos_r = 0, hy_pos_c = 0;
    bool hy_ok = false;
    if (hy_role) {
        const int k = t >> 6, c = t & 63;
        const int hr = y0 + (k == 0 ? -2 : k == 1 ? -1 : k == 2 ? TYB : TYB + 1), hc = x0 + c;
        hy_ok = hr >= 0 && hr <= ny && hc <= nx;
        hy_idx = hr * px + hc + ox;
        hy_pos_r = k == 0 ? 0 : k == 1 ? 1 : k == 2 ? TYB + 2 : TYB + 3;
        hy_pos_c = c + 2;
    }
    // halo D roles: D^x at columns x0-1 / x0+64 for the TYB rows, D^y at rows y0-1 / y0+TYB
    const bool hdx_role = t < 2 * TYB;
    const int hdx_r = t >> 1, hdx_side = t & 1;
    const int hdx_col = hdx_side ? x0 + W : x0 - 1, hdx_row = y0 + hdx_r;
    const int hdx_face = (hdx_role && hdx_row <= ny) ? (hdx_col == 0 ? 0 : hdx_col == nx ? 1 : -1) : -1;
    const bool hdy_role = t < 2 * W;
    const int hdy_side = t >> 6, hdy_c = t & 63;
    const int hdy_row = hdy_side ? y0 + TYB : y0 - 1, hdy_col = x0 + hdy_c;
    const int hdy_face = (hdy_role && hdy_col <= nx) ? (hdy_row == 0 ? 0 : hdy_row == ny ? 1 : -1) : -1;

    auto ldp = [&](int zz, int idx, bool ok) -> C<R> {   // Psi_in at plane zz (block-uniform bounds)
        return (ok && zz >= 0 && zz <= nz) ? cvt<R, IN>(in[zz * plane + idx]) : czero<R>();
    };
    auto d2 = [&](const C<R> &m, const C<R> &c, const C<R> &p) -> C<R> { return d2u<R>(m, c, p); };
    auto dz_at = [&](int zz, const C<R> &m, const C<R> &c, const C<R> &p) -> C<R> {
        if (!col_ok) return czero<R>();
        if (zz == 0) return unscaled<R>(DBz[y * (nx + 1) + x], lc.h2);
        if (zz == nz) return unscaled<R>(DBz[fz + y * (nx + 1) + x], lc.h2);
        return d2(m, c, p);
    };
    struct Ops { C<M> pn; C<R> kt; R vv; };
    auto ld_ops = [&](int zz) -> Ops {
        Ops o;
        o.pn = mk<M>(M(0), M(0));
        o.kt = czero<R>();
        o.vv = R(0);
        if (upd_col && zz < nz) {
            const int p = zz * plane + cidx;
            if (STAGE >= 2 || !in_is_r) o.pn = psin[p];
            if (STAGE >= 2) o.kt = K[p];
            if (V) o.vv = V[p];
        }
        return o;
    };

    C<R> q[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) q[k] = ldp(z0 - 2 + k, cidx, col_ok);
    C<R> hx = ldp(z0, hx_idx, hx_ok), hy = ldp(z0, hy_idx, hy_ok);
    Ops ops = ld_ops(z0);
    C<R> dzm = czero<R>(), dz0 = czero<R>();
    if constexpr (ST != 1) {
        dzm = dz_at(z0 - 1, q[0], q[1], q[2]);
        dz0 = dz_at(z0, q[1], q[2], q[3]);
    }

    for (int zi = 0; zi < TZ; ++zi) {
        const int z = z0 + zi;
        if (z >= nz) break;   // block-uniform
        const bool more = (zi + 1 < TZ) && (z + 1 < nz);
        C<R> q5 = czero<R>(), nhx = czero<R>(), nhy = czero<R>();
        Ops nops{mk<M>(M(0), M(0)), czero<R>(), R(0)};
        if (more) {
            q5 = ldp(z + 3, cidx, col_ok);
            nhx = ldp(z + 1, hx_idx, hx_ok);
            nhy = ldp(z + 1, hy_idx, hy_ok);
            nops = ld_ops(z + 1);
        }
        C<R> dzp = czero<R>();
        if constexpr (ST != 1) dzp = dz_at(z + 1, q[2], q[3], q[4]);
        sp[ty + 2][tx + 2] = q[2];
        if (hx_role) sp[hx_pos_r][hx_pos_c] = hx;
        if (hy_role) sp[hy_pos_r][hy_pos_c] = hy;
        __syncthreads();
        C<R> dx = czero<R>(), dy = czero<R>(), lapnc = czero<R>();
        if constexpr (ST != 1) {
            dx = d2(sp[ty + 2][tx + 1], q[2], sp[ty + 2][tx + 3]);
            dy = d2(sp[ty + 1][tx + 2], q[2], sp[ty + 3][tx + 2]);
        } else if (upd_col) {   // the plane buffer is read before the barrier that lets it be rewritten
            const C<R> u = q[2];
            const R i12h2 = (R)(A.c.ih2 / 12.0);
            const C<R> xm1 = sp[ty + 2][tx + 1], xp1 = sp[ty + 2][tx + 3];
            const C<R> ym1 = sp[ty + 1][tx + 2], yp1 = sp[ty + 3][tx + 2];
            // beyond a face: the ghost carrying the face value D^a_b (h^2-scaled)
            const C<R> xm2 = x == 1 ? ghost<R>(xm1, u, unscaled<R>(DBx[z * (ny + 1) + y], lc.h2)) : sp[ty + 2][tx];
            const C<R> xp2 = x == nx - 1 ? ghost<R>(xp1, u, unscaled<R>(DBx[fx + z * (ny + 1) + y], lc.h2))
                                         : sp[ty + 2][tx + 4];
            const C<R> ym2 = y == 1 ? ghost<R>(ym1, u, unscaled<R>(DBy[z * (nx + 1) + x], lc.h2)) : sp[ty][tx + 2];
            const C<R> yp2 = y == ny - 1 ? ghost<R>(yp1, u, unscaled<R>(DBy[fy + z * (nx + 1) + x], lc.h2))
                                         : sp[ty + 4][tx + 2];
            const C<R> zm2 = z == 1 ? ghost<R>(q[1], u, unscaled<R>(DBz[y * (nx + 1) + x], lc.h2)) : q[0];
            const C<R> zp2 = z == nz - 1 ? ghost<R>(q[3], u, unscaled<R>(DBz[fz + y * (nx + 1) + x], lc.h2)) : q[4];
            lapnc = cadd<R>(cadd<R>(d4nc<R>(xm2, xm1, u, xp1, xp2, i12h2), d4nc<R>(ym2, ym1, u, yp1, yp2, i12h2)),
                            d4nc<R>(zm2, q[1], u, q[3], zp2, i12h2));
        }
        if constexpr (ST == 0) {
            if (xface) dx = unscaled<R>(DBx[fx + z * (ny + 1) + y], lc.h2);
            if (yface) dy = unscaled<R>(DBy[fy + z * (nx + 1) + x], lc.h2);
            sdx[ty][tx + 1] = dx;
            sdy[ty + 1][tx] = dy;
        }
        if (ST == 0 && hdx_role) {
            const int c = hdx_side ? W + 2 : 1;
            C<R> hdx = d2(sp[hdx_r + 2][c - 1], sp[hdx_r + 2][c], sp[hdx_r + 2][c + 1]);
            if (hdx_face >= 0) hdx = unscaled<R>(DBx[hdx_face * fx + z * (ny + 1) + hdx_row], lc.h2);
            sdx[hdx_r][hdx_side ? W + 1 : 0] = hdx;
        }
        if (ST == 0 && hdy_role) {
            const int r = hdy_side ? TYB + 2 : 1;
            C<R> hdy = d2(sp[r - 1][hdy_c + 2], sp[r][hdy_c + 2], sp[r + 1][hdy_c + 2]);
            if (hdy_face >= 0) hdy = unscaled<R>(DBy[hdy_face * fy + z * (nx + 1) + hdy_col], lc.h2);
            sdy[hdy_side ? TYB + 1 : 0][hdy_c] = hdy;
        }
        __syncthreads();
        // The prefetched plane joins the queues, and its loads are waited for (settle), before
        // this plane's stores are issued.
        const C<R> u = q[2], dzm_c = dzm, dz0_c = dz0;
        const Ops cur = ops;
        q[0] = q[1];
        q[1] = q[2];
        q[2] = q[3];
        q[3] = q[4];
        q[4] = q5;
        hx = nhx;
        hy = nhy;
        ops = nops;
        dzm = dz0;
        dz0 = dzp;
        settle(q[4]);
        settle(hx);
        settle(hy);
        if constexpr (STAGE >= 2 || !in_is_r) settle(ops.pn);
        if constexpr (STAGE >= 2) settle(ops.kt);
        settle(ops.vv);
        if (upd_col) {
            const int p = z * plane + cidx;
            C<R> F;
            if constexpr (ST == 0) {
                const C<R> alap = lap3<R>(dx, dy, dz0_c, sdx[ty][tx], sdx[ty][tx + 2], sdy[ty][tx], sdy[ty + 2][tx],
                                          dzm_c, dzp, lc.A76, lc.A112);
                F = rhs_a<R>(alap, u, cur.vv, s);
            } else if constexpr (ST == 2) {   // a/h^2 (D^x + D^y + D^z) from the unscaled differences
                F = rhs_a<R>(cscale<R>((R)(A.c.a * A.c.ih2), cadd<R>(cadd<R>(dx, dy), dz0_c)), u, cur.vv, s);
            } else {
                F = rhs<R>(lapnc, u, cur.vv, (R)A.c.a, s);
            }
            if (STAGE == 1) {
                const C<M> base = in_is_r ? cvt<M, R>(u) : cur.pn;
                K[p] = F;
                out[p] = cvt<R, M>(axpy_m<R, M>(base, ck, F));
            } else if (STAGE <= 3) {
                K[p] = kacc<R>(cur.kt, F);
                out[p] = cvt<R, M>(axpy_m<R, M>(cur.pn, ck, F));
            } else {
                psin[p] = axpy_m<R, M>(cur.pn, ck, cadd<R>(cur.kt, F));
            }
        }
    }
}

template <typename IN, typename R, typename M, int TYB, int TZ, int STAGE, int ST>
static hipError_t launch3(const StageArgs &a, hipStream_t st)
{
    const int64_t tiles_x = (a.L.nx - 1 + 63) / 64;
    const int64_t tiles_y = (a.L.ny - 1 + TYB - 1) / TYB;
    const int64_t tiles_z = (a.L.nz - 1 + TZ - 1) / TZ;
    const int64_t blocks = tiles_x * tiles_y * tiles_z;
    hipLaunchKernelGGL((stage3d_kernel<IN, R, M, TYB, TZ, STAGE, ST>), dim3((unsigned)blocks), dim3(64 * TYB), 0, st, a,
                       (int)tiles_x, (int)tiles_y);
    return hipGetLastError();
}

template <typename IN, typename R, typename M, int TYB, int TZ, int ST>
static hipError_t launch3s(const StageArgs &a, hipStream_t st)
{
    switch (a.stage) {
    case 1: return launch3<IN, R, M, TYB, TZ, 1, ST>(a, st);
    case 2: return launch3<IN, R, M, TYB, TZ, 2, ST>(a, st);
    case 3: return launch3<IN, R, M, TYB, TZ, 3, ST>(a, st);
    default: return launch3<IN, R, M, TYB, TZ, 4, ST>(a, st);
    }
}

template <typename IN, typename R, typename M, int ST>
static hipError_t launch3t(const StageArgs &a, hipStream_t st)
{
    switch (a.variant) {
    case 0: return launch3s<IN, R, M, 4, 32, ST>(a, st);
    case 1: return launch3s<IN, R, M, 4, 64, ST>(a, st);
    case 2: return launch3s<IN, R, M, 8, 32, ST>(a, st);
    case 3: return launch3s<IN, R, M, 4, 16, ST>(a, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename IN, typename R, typename M>
static hipError_t launch3v(const StageArgs &a, hipStream_t st)
{
    switch (a.stencil) {
    case 0: return launch3t<IN, R, M, 0>(a, st);
    case 1: return launch3t<IN, R, M, 1>(a, st);
    case 2: return launch3t<IN, R, M, 2>(a, st);
    default: return hipErrorInvalidValue;
    }
}

int stage3d_variants() { return 4; }

hipError_t launch_stage3d(Prec prec, const StageArgs &a, hipStream_t st)
{
    // 32-bit element offsets: every field (and every face array) must hold < 2^31 elements
    if (a.L.total >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    switch (prec) {
    case P_F64: return launch3v<double, double, double>(a, st);
    case P_F32: return launch3v<float, float, float>(a, st);
    default:
        if (a.stage == 1) return launch3v<double, float, double>(a, st);
        return launch3v<float, float, double>(a, st);
    }
}

}  // namespace nlse
