// One fused RK4-stage tile of the 2D per-axis 2SHOC kernel (shared by the
// stand-alone 2D stage kernel and the batched persistent kernel).  See
// stage2d.hip for the scheme.  Every wave of the block must call this the same
// number of times (waves without a tile pass tile >= tiles_total): it contains
// block-wide barriers.
#pragma once

#include "kernels.h"
#include "point.h"

namespace nlse {

template <typename T, typename U> struct same_t { static constexpr bool v = false; };
template <typename T> struct same_t<T, T> { static constexpr bool v = true; };

constexpr int TILE_W = 64;

// ST selects the Laplacian: 0 the per-axis 2SHOC form, 1 the non-compact fourth-order
// stencil (one node beyond a face the ghost 2 Psi_b - Psi_{b-+1} + h^2 D^a_b, whose second
// difference at b is the face value), 2 the second-order CD.
template <typename IN, typename R, typename M, int RW, int NW, int ST = 0>
__device__ __forceinline__ void stage2d_tile(const StageArgs &A, int64_t tile, int64_t tiles_x, int64_t tiles_total,
                                             C<R> (*lds)[RW][TILE_W + 4], C<R> (*ldx)[RW][TILE_W + 2])
{
    static_assert(RW <= 16, "halo load covers at most 16 rows");
    constexpr int W = TILE_W;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const Layout L = A.L;
    const bool valid = tile < tiles_total;
    const int64_t tx = valid ? tile % tiles_x : 0, ty = valid ? tile / tiles_x : 0;
    const int64_t x0 = 1 + W * tx, y0 = 1 + RW * ty;
    const int64_t x = x0 + lane;
    const bool xnode = valid && x <= L.nx;

    const R a = (R)A.c.a, s = (R)A.c.s;
    const Step2Coef<R> lc = step2_coef<R>(A.c.a, A.c.c76, A.c.c112, A.c.ih2);
    const R ck = (R)A.c.ck;
    const int stage = A.stage;
    const C<IN> *in = (const C<IN> *)A.in;
    const C<R> *DBx = (const C<R> *)A.DB[0];
    const C<R> *DBy = (const C<R> *)A.DB[1];
    const R *V = (const R *)A.V;
    C<M> *psin = (C<M> *)A.psin;
    C<R> *K = (C<R> *)A.K;
    C<R> *out = (C<R> *)A.out;
    constexpr bool in_is_r = same_t<IN, R>::v;

    // ---- global loads: own column rows y0-2 .. y0+RW+1, then the update operands
    C<R> col[RW + 4];
#pragma unroll
    for (int r = 0; r < RW + 4; ++r) {
        const int64_t y = y0 - 2 + r;
        col[r] = czero<R>();
        if (xnode && y >= 0 && y <= L.ny) col[r] = cvt<R, IN>(in[L.idx(x, y, 0)]);
    }
    C<R> hv = czero<R>();
    if (valid && lane < 4 * RW) {
        const int r = lane >> 2, k = lane & 3;
        const int64_t hx = x0 + (k == 0 ? -2 : k == 1 ? -1 : k == 2 ? W : W + 1);
        const int64_t y = y0 + r;
        if (hx >= 0 && hx <= L.nx && y <= L.ny) hv = cvt<R, IN>(in[L.idx(hx, y, 0)]);
    }
    C<M> pn[RW];
    C<R> kt[RW];
    R vv[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int64_t y = y0 + r;
        const bool upd = xnode && x < L.nx && y < L.ny;
        const int64_t p = L.idx(x, y, 0);
        pn[r] = mk<M>(M(0), M(0));
        kt[r] = czero<R>();
        vv[r] = R(0);
        if (upd && (stage >= 2 || !in_is_r)) pn[r] = psin[p];
        if (upd && stage >= 2) kt[r] = K[p];
        if (upd && V) vv[r] = V[p];
    }

    // ---- step 1 along x: Psi row (+ halo) through LDS
#pragma unroll
    for (int r = 0; r < RW; ++r) lds[wv][r][lane + 2] = col[r + 2];
    if (lane < 4 * RW) {
        const int r = lane >> 2, k = lane & 3;
        lds[wv][r][k == 0 ? 0 : k == 1 ? 1 : k == 2 ? W + 2 : W + 3] = hv;
    }
    __syncthreads();
    C<R> dx[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        dx[r] = d2u<R>(lds[wv][r][lane + 1], lds[wv][r][lane + 2], lds[wv][r][lane + 3]);
        if (xnode && x == L.nx && y0 + r <= L.ny) dx[r] = unscaled<R>(DBx[(L.ny + 1) + y0 + r], lc.h2);   // face x = nx
    }
#pragma unroll
    for (int r = 0; r < RW; ++r) ldx[wv][r][lane + 1] = dx[r];
    if (valid && lane < 2 * RW) {
        const int r = lane >> 1, side = lane & 1;
        const int c = side ? W + 2 : 1;               // LDS column of x0+64 or x0-1
        C<R> hdx = d2u<R>(lds[wv][r][c - 1], lds[wv][r][c], lds[wv][r][c + 1]);
        const int64_t hx = side ? x0 + W : x0 - 1;
        const int64_t y = y0 + r;
        if (y <= L.ny) {
            if (hx == 0) hdx = unscaled<R>(DBx[y], lc.h2);
            else if (hx == L.nx) hdx = unscaled<R>(DBx[(L.ny + 1) + y], lc.h2);
        }
        ldx[wv][r][side ? W + 1 : 0] = hdx;
    }

    // ---- step 1 along y: registers
    C<R> dy[RW + 2];
#pragma unroll
    for (int j = 0; j < RW + 2; ++j) {
        const int64_t y = y0 - 1 + j;
        dy[j] = d2u<R>(col[j], col[j + 1], col[j + 2]);
        if (xnode && y == 0) dy[j] = unscaled<R>(DBy[x], lc.h2);
        if (xnode && y == L.ny) dy[j] = unscaled<R>(DBy[(L.nx + 1) + x], lc.h2);
    }
    __syncthreads();

    // ---- step 2, F and the RK4 stage update
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int64_t y = y0 + r;
        if (!(xnode && x < L.nx && y < L.ny)) continue;
        const C<R> u = col[r + 2];
        C<R> F;
        if constexpr (ST == 0) {
            const C<R> alap = lap2a<R>(dx[r], dy[r + 1], ldx[wv][r][lane], ldx[wv][r][lane + 2], dy[r], dy[r + 2],
                                       lc.A76, lc.A112);
            F = rhs_a<R>(alap, u, vv[r], s);
        } else if constexpr (ST == 2) {   // a/h^2 (D^x + D^y) from the unscaled differences
            F = rhs_a<R>(cscale<R>((R)(A.c.a * A.c.ih2), cadd<R>(dx[r], dy[r + 1])), u, vv[r], s);
        } else {
            const R i12h2 = (R)(A.c.ih2 / 12.0);
            const C<R> c = col[r + 2];
            const C<R> xm1 = lds[wv][r][lane + 1], xp1 = lds[wv][r][lane + 3];
            const C<R> ym1 = col[r + 1], yp1 = col[r + 3];
            // beyond a face: the ghost carrying the face value D^a_b (h^2-scaled)
            const C<R> xm2 = x == 1 ? ghost<R>(xm1, c, unscaled<R>(DBx[y], lc.h2)) : lds[wv][r][lane];
            const C<R> xp2 = x == L.nx - 1 ? ghost<R>(xp1, c, unscaled<R>(DBx[(L.ny + 1) + y], lc.h2))
                                           : lds[wv][r][lane + 4];
            const C<R> ym2 = y == 1 ? ghost<R>(ym1, c, unscaled<R>(DBy[x], lc.h2)) : col[r];
            const C<R> yp2 = y == L.ny - 1 ? ghost<R>(yp1, c, unscaled<R>(DBy[(L.nx + 1) + x], lc.h2)) : col[r + 4];
            const C<R> lap = cadd<R>(d4nc<R>(xm2, xm1, c, xp1, xp2, i12h2), d4nc<R>(ym2, ym1, c, yp1, yp2, i12h2));
            F = rhs<R>(lap, u, vv[r], a, s);
        }
        const int64_t p = L.idx(x, y, 0);
        if (stage == 1) {
            const C<M> base = in_is_r ? cvt<M, R>(u) : pn[r];
            K[p] = F;
            out[p] = cvt<R, M>(axpy_m<R, M>(base, ck, F));
        } else if (stage <= 3) {
            K[p] = kacc<R>(kt[r], F);
            out[p] = cvt<R, M>(axpy_m<R, M>(pn[r], ck, F));
        } else {
            psin[p] = axpy_m<R, M>(pn[r], ck, cadd<R>(kt[r], F));
        }
    }
}

}  // namespace nlse
