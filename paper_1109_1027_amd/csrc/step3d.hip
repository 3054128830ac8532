// Two fused RK4 stages per launch for the 3D NLSE with the per-axis 2SHOC
// Laplacian (Sec. 2.3 Eqs. 3d2shocMs1-2, Sec. 3.1 Eq. RK4).
//
// One RK4 step is two launches:
//   pair 1  stages 1 and 2: reads Psi^n and V; writes K = F1 + 2 F2 and the
//           stage field B = Psi^n + (k/2) F2;
//   pair 2  stages 3 and 4: reads B, K, Psi^n and V; writes
//           Psi^{n+1} = Psi^n + (k/6)(K + 2 F3 + F4) into a second master buffer
//           (its neighbours still read Psi^n, so the update cannot be in place).
// Against four stage launches this never writes the stage-1 and stage-3 fields
// and never reads them back: 64 B per point and step instead of 152 in FP32.
//
// Scheme.  A block owns a thread tile of 64 x TY columns and marches along z.
// The first stage of the pair (alpha) is evaluated on every column of the tile,
// exactly as the stage kernel evaluates its tile (the input plane with a
// two-node halo in LDS, D^x and D^y with a one-node halo, D^z from the column's
// own queue); its result stays on chip: a five-plane queue per column and, one
// plane at a time, LDS.  The second stage (beta) needs alpha's field two nodes
// around each of its points, so it produces only the inner 60 x (TY - 4)
// columns: tiles overlap by four columns and four rows.  Along z the stages
// are skewed: when input plane z arrives, alpha produces plane z - 2 and beta
// plane z - 4.  Alpha's field waits in a three-plane LDS ring, so beta's
// in-plane differences at plane z - 4 are formed in the same phase as alpha's at
// z - 2: two barriers per plane (input plane written / all D^x, D^y written).
//
// The point-wise arithmetic is the stage kernel's (point.h), so the fields are
// bit-identical to four stage launches.  Face closure values D^a_b are the
// Dirichlet constants of launch_boundary_d (Dirichlet only).
#include "kernels.h"
#include "point.h"

namespace nlse {

namespace {

template <typename T, typename U> struct same_p { static constexpr bool v = false; };
template <typename T> struct same_p<T, T> { static constexpr bool v = true; };

constexpr int PW = 64;          // thread-tile width: one wave per row

constexpr int OXW = PW - 4;     // output columns per tile

template <typename IN, typename R, typename M, int TY, int TZ, int PAIR>
__global__ __launch_bounds__(PW * TY) void pair3d_kernel(Step3DArgs A, int tiles_x, int tiles_y)
{
    static_assert(TY >= 8 && PW * TY >= 4 * PW, "halo roles need at least 256 threads");
    constexpr int OY = TY - 4;
    __shared__ C<R> sp[TY + 4][PW + 4];   // a plane of alpha's input, columns xs-2 .. xs+65
    __shared__ C<R> sdx[TY][PW + 2];      // alpha's D^x, columns xs-1 .. xs+64
    __shared__ C<R> sdy[TY + 2][PW];      // alpha's D^y, rows ys-1 .. ys+TY
    __shared__ C<R> sa[3][TY][PW];        // alpha's field, planes za, za-1, za-2 (plane q in slot q mod 3)
    __shared__ C<R> sbx[TY][PW];          // beta's D^x and D^y
    __shared__ C<R> sby[TY][PW];

    const int t = threadIdx.x, tx = t & 63, ty = t >> 6;
    const int nx = (int)A.L.nx, ny = (int)A.L.ny, nz = (int)A.L.nz;
    const int px = (int)A.L.px, ox = (int)A.L.ox;
    const int plane = px * (int)A.L.py;
    const int lb = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % tiles_x, by = (lb / tiles_x) % tiles_y, bz = lb / (tiles_x * tiles_y);
    const int xs = OXW * bx - 1, ys = OY * by - 1;          // column of thread (0, 0)
    const int z0 = 1 + TZ * bz, z1 = min(z0 + TZ, nz) - 1;  // output planes z0 .. z1
    const int x = xs + tx, y = ys + ty;
    const bool col_in = x >= 0 && x <= nx && y >= 0 && y <= ny;
    const bool col_int = x >= 1 && x < nx && y >= 1 && y < ny;
    const bool col_out = col_int && tx >= 2 && tx < PW - 2 && ty >= 2 && ty < TY - 2;
    const int cidx = col_in ? y * px + x + ox : 0;          // own column, plane 0
    const int fzi = col_in ? y * (nx + 1) + x : 0;          // own column in the z faces
    // The tile's threads touch a boundary face (block-uniform): only then do they read face values.
    const bool tile_face = xs <= 1 || xs + PW >= nx || ys <= 1 || ys + TY >= ny;

    const R s = (R)A.c.s;
    const Step2Coef<R> lc = step2_coef<R>(A.c.a, A.c.c76, A.c.c112, A.c.ih2);   // 1/h^2 and a folded in
    const R ck_a = (R)A.ck[PAIR == 1 ? 0 : 2], ck_b = (R)A.ck[PAIR == 1 ? 1 : 3];
    const C<IN> *in = PAIR == 1 ? (const C<IN> *)A.psin : (const C<IN> *)A.B;
    const C<M> *psin = (const C<M> *)A.psin;
    const C<R> *DBx = (const C<R> *)A.DB[0];
    const C<R> *DBy = (const C<R> *)A.DB[1];
    const C<R> *DBz = (const C<R> *)A.DB[2];
    const R *V = (const R *)A.V;
    const C<R> *Kin = (const C<R> *)A.K;
    C<R> *Kout = (C<R> *)A.K;
    C<R> *Bout = (C<R> *)A.B;
    C<M> *pout = (C<M> *)A.psi_out;
    const int fx = (nz + 1) * (ny + 1), fy = (nz + 1) * (nx + 1), fz = (ny + 1) * (nx + 1);

    // halo roles, fixed for the whole march (as in the stage kernel)
    const bool hx_role = t < 4 * TY;
    int hx_idx = 0, hx_pos_r = 0, hx_pos_c = 0;
    bool hx_ok = false;
    if (hx_role) {
        const int r = t >> 2, k = t & 3;
        const int hc = xs + (k == 0 ? -2 : k == 1 ? -1 : k == 2 ? PW : PW + 1), hr = ys + r;
        hx_ok = hc >= 0 && hc <= nx && hr >= 0 && hr <= ny;
        hx_idx = hx_ok ? hr * px + hc + ox : 0;
        hx_pos_r = r + 2;
        hx_pos_c = k == 0 ? 0 : k == 1 ? 1 : k == 2 ? PW + 2 : PW + 3;
    }
    const bool hy_role = t < 4 * PW;
    int hy_idx = 0, hy_pos_r = 0, hy_pos_c = 0;
    bool hy_ok = false;
    if (hy_role) {
        const int k = t >> 6, c = t & 63;
        const int hr = ys + (k == 0 ? -2 : k == 1 ? -1 : k == 2 ? TY : TY + 1), hc = xs + c;
        hy_ok = hr >= 0 && hr <= ny && hc >= 0 && hc <= nx;
        hy_idx = hy_ok ? hr * px + hc + ox : 0;
        hy_pos_r = k == 0 ? 0 : k == 1 ? 1 : k == 2 ? TY + 2 : TY + 3;
        hy_pos_c = c + 2;
    }
    // D^x at columns xs-1 / xs+64 for the TY rows, D^y at rows ys-1 / ys+TY
    const bool hdx_role = t < 2 * TY;
    const int hdx_r = t >> 1, hdx_side = t & 1;
    const int hdx_col = hdx_side ? xs + PW : xs - 1, hdx_row = ys + hdx_r;
    const bool hdx_in = hdx_role && hdx_row >= 0 && hdx_row <= ny;
    const int hdx_face = hdx_in ? (hdx_col == 0 ? 0 : hdx_col == nx ? 1 : -1) : -1;
    const bool hdy_role = t < 2 * PW;
    const int hdy_side = t >> 6, hdy_c = t & 63;
    const int hdy_row = hdy_side ? ys + TY : ys - 1, hdy_col = xs + hdy_c;
    const bool hdy_in = hdy_role && hdy_col >= 0 && hdy_col <= nx;
    const int hdy_face = hdy_in ? (hdy_row == 0 ? 0 : hdy_row == ny ? 1 : -1) : -1;

    // Loads are unconditional, from a plane clamped into the grid (every idx above is a valid
    // node of a plane), and the value is then selected: a branch around a load costs scalar
    // exec-mask work on every plane and waits for every load in flight where it joins.
    auto ldi = [&](int zz, int idx, bool ok) -> C<IN> {   // stage input at plane zz
        const C<IN> v = in[min(max(zz, 0), nz) * plane + idx];
        return (ok && zz >= 0 && zz <= nz) ? v : mk<IN>(IN(0), IN(0));
    };
    // D^z from three planes of a column, or the z-face value on a boundary plane
    auto dz_at = [&](int zz, const C<R> &m, const C<R> &c, const C<R> &p) -> C<R> {
        C<R> d = d2u<R>(m, c, p);
        if (zz == 0 || zz == nz) d = unscaled<R>(DBz[(zz == 0 ? 0 : fz) + fzi], lc.h2);   // block-uniform
        return (col_in && zz >= 0 && zz <= nz) ? d : czero<R>();
    };
    struct Ops { C<M> pn; C<R> kt; R vv; };   // alpha's update operands at one plane
    auto ld_ops = [&](int zz) -> Ops {
        const bool ok = col_int && zz >= 1 && zz < nz;
        const int p = min(max(zz, 1), nz - 1) * plane + cidx;
        Ops o{mk<M>(M(0), M(0)), czero<R>(), R(0)};
        if (PAIR == 2) {
            const C<M> pn = psin[p];
            const C<R> kt = Kin[p];
            if (ok) {
                o.pn = pn;
                o.kt = kt;
            }
        }
        if (V) {
            const R vv = V[p];
            if (ok) o.vv = vv;
        }
        return o;
    };

    // ---- prologue: input planes z0-4 .. z0, D^z_alpha at z0-3 and z0-2, halo of plane z0-2
    C<IN> qi[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) qi[k] = ldi(z0 - 4 + k, cidx, col_in);
    C<R> dza[3];   // D^z of the alpha input at planes za-1, za, za+1
    dza[0] = czero<R>();
    dza[1] = dz_at(z0 - 3, cvt<R, IN>(qi[0]), cvt<R, IN>(qi[1]), cvt<R, IN>(qi[2]));
    dza[2] = dz_at(z0 - 2, cvt<R, IN>(qi[1]), cvt<R, IN>(qi[2]), cvt<R, IN>(qi[3]));
    C<R> hx = cvt<R, IN>(ldi(z0 - 2, hx_idx, hx_ok)), hy = cvt<R, IN>(ldi(z0 - 2, hy_idx, hy_ok));
    Ops ops = ld_ops(z0 - 2);
    C<R> qa[5];    // alpha's field at planes za-4 .. za
    C<R> dzb[3];   // D^z of alpha's field at planes zb-1, zb, zb+1
    C<R> kq[3];    // K after alpha at planes za, za-1, za-2
    C<M> pq[3];    // Psi^n at planes za, za-1, za-2 (pair 2; pair 1 reads it from qi)
    R vq[3];       // V at planes za, za-1, za-2
#pragma unroll
    for (int k = 0; k < 5; ++k) qa[k] = czero<R>();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dzb[k] = kq[k] = czero<R>();
        pq[k] = mk<M>(M(0), M(0));
        vq[k] = R(0);
    }

    for (int zi = z0; zi <= z1 + 4; ++zi) {   // block-uniform bounds
        const int za = zi - 2, zb = zi - 4;
        // prefetch what plane za + 1 needs
        const C<IN> qn = ldi(zi + 1, cidx, col_in);
        const C<R> nhx = cvt<R, IN>(ldi(za + 1, hx_idx, hx_ok)), nhy = cvt<R, IN>(ldi(za + 1, hy_idx, hy_ok));
        const Ops nops = ld_ops(za + 1);

        // ---- alpha at plane za on every column of the tile
        dza[0] = dza[1];
        dza[1] = dza[2];
        dza[2] = dz_at(za + 1, cvt<R, IN>(qi[2]), cvt<R, IN>(qi[3]), cvt<R, IN>(qi[4]));
        const C<R> u = cvt<R, IN>(qi[2]);
        sp[ty + 2][tx + 2] = u;
        if (hx_role) sp[hx_pos_r][hx_pos_c] = hx;
        if (hy_role) sp[hy_pos_r][hy_pos_c] = hy;
        __syncthreads();
        const bool zin = za >= 0 && za <= nz;   // block-uniform
        const bool beta = zb >= z0;             // block-uniform
        C<R> bdx = czero<R>(), bdy = czero<R>();
        if (beta) {   // beta's in-plane differences at plane zb, from alpha's field two planes back
            const C<R>(*pa)[PW] = sa[(zb + 3) % 3];
            const int xl = max(tx - 1, 0), xr = min(tx + 1, PW - 1), yl = max(ty - 1, 0), yr = min(ty + 1, TY - 1);
            const C<R> ub = pa[ty][tx];
            bdx = d2u<R>(pa[ty][xl], ub, pa[ty][xr]);   // tile-border threads: unused
            bdy = d2u<R>(pa[yl][tx], ub, pa[yr][tx]);
            if (tile_face && col_in) {   // zb lies in 1 .. nz-1
                if (x == 0) bdx = unscaled<R>(DBx[zb * (ny + 1) + y], lc.h2);
                else if (x == nx) bdx = unscaled<R>(DBx[fx + zb * (ny + 1) + y], lc.h2);
                if (y == 0) bdy = unscaled<R>(DBy[zb * (nx + 1) + x], lc.h2);
                else if (y == ny) bdy = unscaled<R>(DBy[fy + zb * (nx + 1) + x], lc.h2);
            }
            sbx[ty][tx] = bdx;
            sby[ty][tx] = bdy;
        }
        C<R> dx = d2u<R>(sp[ty + 2][tx + 1], u, sp[ty + 2][tx + 3]);
        C<R> dy = d2u<R>(sp[ty + 1][tx + 2], u, sp[ty + 3][tx + 2]);
        if (tile_face && col_in && zin) {
            if (x == 0) dx = unscaled<R>(DBx[za * (ny + 1) + y], lc.h2);
            else if (x == nx) dx = unscaled<R>(DBx[fx + za * (ny + 1) + y], lc.h2);
            if (y == 0) dy = unscaled<R>(DBy[za * (nx + 1) + x], lc.h2);
            else if (y == ny) dy = unscaled<R>(DBy[fy + za * (nx + 1) + x], lc.h2);
        }
        sdx[ty][tx + 1] = dx;
        sdy[ty + 1][tx] = dy;
        if (hdx_role) {
            const int c = hdx_side ? PW + 2 : 1;
            C<R> hdx = d2u<R>(sp[hdx_r + 2][c - 1], sp[hdx_r + 2][c], sp[hdx_r + 2][c + 1]);
            if (tile_face && hdx_face >= 0 && zin) hdx = unscaled<R>(DBx[hdx_face * fx + za * (ny + 1) + hdx_row], lc.h2);
            sdx[hdx_r][hdx_side ? PW + 1 : 0] = hdx;
        }
        if (hdy_role) {
            const int r = hdy_side ? TY + 2 : 1;
            C<R> hdy = d2u<R>(sp[r - 1][hdy_c + 2], sp[r][hdy_c + 2], sp[r + 1][hdy_c + 2]);
            if (tile_face && hdy_face >= 0 && zin) hdy = unscaled<R>(DBy[hdy_face * fy + za * (nx + 1) + hdy_col], lc.h2);
            sdy[hdy_side ? TY + 1 : 0][hdy_c] = hdy;
        }
        __syncthreads();
        C<R> ua = u, ka = czero<R>();   // alpha's field (boundary: unchanged) and K after alpha
        if (za >= 1 && za < nz) {   // block-uniform; every lane computes, interior lanes keep it
            const C<R> alap = lap3<R>(dx, dy, dza[1], sdx[ty][tx], sdx[ty][tx + 2], sdy[ty][tx], sdy[ty + 2][tx],
                                      dza[0], dza[2], lc.A76, lc.A112);
            const C<R> F = rhs_a<R>(alap, u, ops.vv, s);
            C<R> kn, un;
            if (PAIR == 1) {   // stage 1: K = F, field Psi^n + (k/2) F
                kn = F;
                un = cvt<R, M>(axpy_m<R, M>(cvt<M, IN>(qi[2]), ck_a, F));
            } else {           // stage 3: K += 2F, field Psi^n + k F
                kn = kacc<R>(ops.kt, F);
                un = cvt<R, M>(axpy_m<R, M>(ops.pn, ck_a, F));
            }
            if (col_int) {
                ka = kn;
                ua = un;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) qa[k] = qa[k + 1];
        qa[4] = ua;
        kq[2] = kq[1];
        kq[1] = kq[0];
        kq[0] = ka;
        if constexpr (PAIR == 2) {
            pq[2] = pq[1];
            pq[1] = pq[0];
            pq[0] = ops.pn;
        }
        vq[2] = vq[1];
        vq[1] = vq[0];
        vq[0] = ops.vv;
        dzb[0] = dzb[1];
        dzb[1] = dzb[2];
        dzb[2] = dz_at(za - 1, qa[2], qa[3], qa[4]);
        if (za >= z0 - 2) sa[(za + 3) % 3][ty][tx] = ua;   // for beta two planes on (slot of plane za - 3)

        // The prefetched plane joins the queues, and its loads are waited for (settle), before
        // beta's stores are issued.
        const C<IN> q_zb = qi[0];   // Psi^n at zb (pair 1)
#pragma unroll
        for (int k = 0; k < 4; ++k) qi[k] = qi[k + 1];
        qi[4] = qn;
        hx = nhx;
        hy = nhy;
        ops = nops;
        settle(qi[4]);
        settle(hx);
        settle(hy);
        if constexpr (PAIR == 2) {
            settle(ops.pn);
            settle(ops.kt);
        }
        settle(ops.vv);
        // ---- beta at plane zb on the inner columns
        if (beta) {
            const C<R> ub = qa[2];
            if (col_out) {
                const C<R> alap = lap3<R>(bdx, bdy, dzb[1], sbx[ty][tx - 1], sbx[ty][tx + 1], sby[ty - 1][tx],
                                          sby[ty + 1][tx], dzb[0], dzb[2], lc.A76, lc.A112);
                const C<R> F = rhs_a<R>(alap, ub, vq[2], s);
                const int p = zb * plane + cidx;
                if (PAIR == 1) {   // stage 2: K += 2F, B = Psi^n + (k/2) F
                    Kout[p] = kacc<R>(kq[2], F);
                    Bout[p] = cvt<R, M>(axpy_m<R, M>(cvt<M, IN>(q_zb), ck_b, F));
                } else {           // stage 4: Psi^{n+1} = Psi^n + (k/6)(K + F)
                    pout[p] = axpy_m<R, M>(pq[2], ck_b, cadd<R>(kq[2], F));
                }
            }
        }
        // The next plane writes sp before its first barrier (every read of sp came before this
        // plane's second barrier) and sdx, sdy, sbx, sby only after it; alpha's field goes to
        // slot za mod 3 after the second barrier, while beta read slot zb mod 3 before it.
    }
}

template <typename IN, typename R, typename M, int TY, int TZ, int PAIR>
hipError_t launch_p(const Step3DArgs &a, hipStream_t st)
{
    const int64_t tiles_x = (a.L.nx - 1 + OXW - 1) / OXW;
    const int64_t tiles_y = (a.L.ny - 1 + (TY - 4) - 1) / (TY - 4);
    const int64_t tiles_z = (a.L.nz - 1 + TZ - 1) / TZ;
    const int64_t blocks = tiles_x * tiles_y * tiles_z;
    hipLaunchKernelGGL((pair3d_kernel<IN, R, M, TY, TZ, PAIR>), dim3((unsigned)blocks), dim3(PW * TY), 0, st, a,
                       (int)tiles_x, (int)tiles_y);
    return hipGetLastError();
}

template <typename R, typename M, int TY, int TZ>
hipError_t launch_pairs(const Step3DArgs &a, hipStream_t st)
{
    hipError_t e = launch_p<M, R, M, TY, TZ, 1>(a, st);
    if (e != hipSuccess) return e;
    return launch_p<R, R, M, TY, TZ, 2>(a, st);
}

template <typename R, typename M>
hipError_t launch_v3(const Step3DArgs &a, hipStream_t st)
{
    switch (a.variant) {
    case 0: return launch_pairs<R, M, 16, 32>(a, st);
    case 1: return launch_pairs<R, M, 16, 64>(a, st);
    case 2: return launch_pairs<R, M, 8, 32>(a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int step3d_variants() { return 3; }

hipError_t launch_step3d(Prec prec, const Step3DArgs &a, hipStream_t st)
{
    // 32-bit element offsets: every field (and every face array) must hold < 2^31 elements
    if (a.L.total >= (int64_t(1) << 31) || a.L.dim != 3) return hipErrorInvalidValue;
    switch (prec) {
    case P_F64: return launch_v3<double, double>(a, st);
    case P_F32: return launch_v3<float, float>(a, st);
    default: return launch_v3<float, double>(a, st);
    }
}

}  // namespace nlse
