// One wave's share of the 2D whole-step RK4 kernel (shared by the stand-alone
// whole-step kernel of step2d.hip and the batched persistent kernel): the wave
// advances the interior of one (48-column strip, row segment) task of Psi^n to
// Psi^{n+1}.  See step2d.hip for the scheme.  Contains no barrier; the caller
// provides the wave's private LDS staging for the boundary-face values.
#pragma once

#include "kernels.h"
#include "point.h"
#include "dpp.h"

#include <type_traits>

namespace nlse {
namespace wave2d {

constexpr int SW = 48;     // output columns per strip
constexpr int HALO = 8;    // two rows (columns) per stage

template <int Q> constexpr int seg_rows() { return 9 * Q - 2 * HALO; }   // output rows per segment
template <int Q> constexpr int face_rows() { return 9 * Q + HALO; }      // rows jb-8 .. jb+9Q-1

__host__ __device__ inline int strips(int64_t nx) { return (int)((nx - 1 + SW - 1) / SW); }
template <int Q> __host__ __device__ inline int segments(int64_t ny) { return (int)((ny - 1 + seg_rows<Q>() - 1) / seg_rows<Q>()); }

constexpr int RP = 2;               // zero entries on each side of a ring row
constexpr int RS = 64 + 2 * RP;     // ring row stride

// A wave's private LDS, rewritten by every call.
//   sdx: D^x on the faces x = 0 and x = nx for the task's rows,
//   sdy: D^y on the faces y = 0 and y = ny for its columns,
//   ring: the last three input rows of each stage, lane l at entry l + RP; the entries
//         beyond the wave read zero, as the lanes shifted in by a DPP wave shift do.
template <typename R, int Q>
struct Staging {
    C<R> sdx[2][face_rows<Q>()];
    C<R> sdy[2][64];
    C<R> ring[4][3][RS];
};

// Orders the wave's LDS accesses on either side for the compiler.  Lanes exchange values
// through the staging (a lane reads what its neighbours wrote), which the per-thread view of
// the program does not see as a dependence; the LDS executes one wave's accesses in issue
// order, so keeping the issue order is all the exchange needs.
__device__ __forceinline__ void lds_order()
{
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// strip < strips(nx) and seg < segments<Q>(ny), wave-uniform; the field has < 2^31 elements.
// ST selects the Laplacian as in the stage kernels: 0 the per-axis 2SHOC form, 1 the
// non-compact five-point stencil (ghosts 2 Psi_b - Psi_{b-+1} + h^2 D^a_b beyond a face), 2 the
// second-order CD.
template <typename R, typename M, int Q, int PD = 1, int ST = 0>
__device__ __forceinline__ void step2d_wave(const Step2DArgs &A, int strip, int seg, int lane, Staging<R, Q> &S)
{
    auto &sdx = S.sdx;
    auto &sdy = S.sdy;
    auto &ring = S.ring;
    constexpr int SEG = seg_rows<Q>();
    constexpr int FR = face_rows<Q>();
    lds_order();        // earlier reads of the staging come first
    const int nx = (int)A.L.nx, ny = (int)A.L.ny, px = (int)A.L.px, ox = (int)A.L.ox;
    const int xs = 1 + SW * strip - HALO;   // column of lane 0
    const int x = xs + lane;
    const bool xin = x >= 0 && x <= nx;
    const bool xint = x >= 1 && x < nx;
    const bool xface = x == 0 || x == nx;
    const bool wlane = xint && lane >= HALO && lane < HALO + SW;
    const bool has_face = xs <= 0 || xs + 63 >= nx;   // wave-uniform
    // The task stores rows ys .. y1-1.  Its window of rows starts at y0 = ys, except in the last
    // segment, whose window ends at the face (y0 = ny - SEG, overlapping the segment before it):
    // then the face rows meet the pipeline only in the last group.
    const int ys = 1 + SEG * seg, y1 = min(ys + SEG, ny);
    const int y0 = seg == segments<Q>(ny) - 1 ? max(1, ny - SEG) : ys;
    const int jb = y0 - HALO;               // row of Psi^n that enters at t = 0

    const R s = (R)A.c.s;
    const Step2Coef<R> lc = step2_coef<R>(A.c.a, A.c.c76, A.c.c112, A.c.ih2);
    // The stage updates of stages 1-3 use ck times 1 on interior columns and times 0 elsewhere:
    // Psi^n + 0 * F is Psi^n exactly, so boundary and outside columns keep their values
    // (Eq. dbc_ut) without a select (F is finite there: every value those lanes see is a copy
    // of a field value).  Rows are handled the same way with a wave-uniform factor.
    R ck[4], ckl[3];
#pragma unroll
    for (int i = 0; i < 4; ++i) ck[i] = (R)A.ck[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) ckl[i] = xint ? ck[i] : R(0);
    const C<M> *__restrict__ pin = (const C<M> *)A.psi_in;
    C<M> *__restrict__ pout = (C<M> *)A.psi_out;
    const R *__restrict__ V = (const R *)A.V;
    const C<R> *__restrict__ DBx = (const C<R> *)A.DB[0];
    const C<R> *__restrict__ DBy = (const C<R> *)A.DB[1];

    sdy[0][lane] = xin ? unscaled<R>(DBy[x], lc.h2) : czero<R>();   // unscaled, like d2u
    sdy[1][lane] = xin ? unscaled<R>(DBy[nx + 1 + x], lc.h2) : czero<R>();
    if (has_face) {
        for (int i = lane; i < FR; i += 64) {
            const int r = jb - HALO + i;
            const bool ok = r >= 0 && r <= ny;
            sdx[0][i] = ok ? unscaled<R>(DBx[r], lc.h2) : czero<R>();
            sdx[1][i] = ok ? unscaled<R>(DBx[ny + 1 + r], lc.h2) : czero<R>();
        }
    }
    if (lane < 2 * RP) {
        const int e = lane < RP ? lane : RS - 2 * RP + lane;
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int q = 0; q < 3; ++q) ring[st][q][e] = czero<R>();
    }
    lds_order();

    C<R> U[4][3], D[4][3], Kq[9];
    C<R> Uq[4][5];   // non-compact stencil: each stage's input rows m-4 .. m (a shift queue)
    C<M> P[9];
    R Vq[9];
    const R aR = (R)A.c.a, i12h2 = (R)(A.c.ih2 / 12.0), aih2 = (R)(A.c.a * A.c.ih2);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        Kq[i] = czero<R>();
        P[i] = mk<M>(M(0), M(0));
        Vq[i] = R(0);
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
#pragma unroll
        for (int i = 0; i < 3; ++i) U[st][i] = D[st][i] = czero<R>();
#pragma unroll
        for (int i = 0; i < 5; ++i) Uq[st][i] = czero<R>();
    }

    // Row loads are unconditional, with the address clamped into the field: the
    // number of loads in flight never depends on the path, so waiting for a
    // prefetched row leaves the next row's loads outstanding.  Lanes and rows
    // outside the grid thus hold copies of edge values; they feed no interior
    // node (the face closures replace every D they would enter).
    const int xc = min(max(x, 0), nx);
    auto load_row = [&](int y, C<M> &pv, R &vv) {
        const int o = min(max(y, 0), ny) * px + xc + ox;
        pv = pin[o];
        vv = V[o];
    };
    // PD rows of Psi^n and V in flight ahead of the row being consumed
    C<M> pf[PD];
    R vf[PD];
#pragma unroll
    for (int d = 0; d < PD; ++d) load_row(jb + d, pf[d], vf[d]);

    // One group of nine rows.  A PLAIN group needs none of the tests of the general one: it holds
    // no row t < 16 (where a stage's output is skipped while its inputs are still filling the
    // pipeline, t < 4 (st + 1)), no stage meets a face row (m - 1 = 0 or ny), every output row
    // r lies in 1 .. ny-1 and below y1, and the face columns take their values by a select.
    // That holds for g >= 2 when the newest row of stage 1 stays below the face,
    // jb + 9 g + 8 <= ny.
    auto group = [&](const int g, auto plain_t) {
        constexpr bool plain = decltype(plain_t)::value;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
            const int t = 9 * g + p;
            const int j = jb + t;
            // Ring rows read in this row were written two rows ago; within the row, reads and
            // writes use different ring slots.
            lds_order();
            P[p] = pf[0];
            Vq[p] = vf[0];
#pragma unroll
            for (int d = 0; d + 1 < PD; ++d) {
                pf[d] = pf[d + 1];
                vf[d] = vf[d + 1];
            }
            load_row(j + PD, pf[PD - 1], vf[PD - 1]);   // prefetch
            const int q0 = p % 3, q1 = (p + 1) % 3, q2 = (p + 2) % 3;   // rows m, m-2, m-1
            // face values of the four stages' output rows j-2-2st, read before the stages so
            // that no stage waits for its LDS read (the indices stay inside the staging)
            C<R> fv[4];
            if (has_face) {
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const int i = t + HALO - 2 - 2 * st;
                    if (x == (ST == 1 ? 1 : 0)) fv[st] = sdx[0][i];
                    else fv[st] = sdx[1][i];
                }
            }
            C<R> in = cvt<R, M>(P[p]);
            // x neighbours of the row each stage differentiates (row m-2, written two rows
            // ago): read one stage ahead, before this row's ring writes
            auto read_nb = [&](int st, C<R>(&nb)[4]) {
                const C<R> *row = ring[st][q1] + RP + lane;
                nb[1] = row[-1];
                nb[2] = row[1];
                if constexpr (ST == 1) {
                    nb[0] = row[-2];
                    nb[3] = row[2];
                }
            };
            C<R> nb[4] = {}, nbn[4] = {};
            read_nb(0, nb);
            ring[0][q0][RP + lane] = in;
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                if (st < 3) read_nb(st + 1, nbn);
                const int m = j - 2 * st;   // newest input row of this stage
                if constexpr (ST == 1) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) Uq[st][i] = Uq[st][i + 1];
                    Uq[st][4] = in;
                } else {
                    U[st][q0] = in;
                    C<R> dy = d2u<R>(U[st][q1], U[st][q2], U[st][q0]);   // h^2 D^y at row m-1
                    if (!plain) {
                        if (m - 1 == 0) dy = sdy[0][lane];
                        if (m - 1 == ny) dy = sdy[1][lane];
                    }
                    D[st][q0] = dy;
                }
                C<R> outv = czero<R>();
                if (plain || t >= 4 * (st + 1)) {    // earlier output rows feed nothing
                    const int r = m - 2;    // output row
                    const int kr = (p + 18 - 2 * (st + 1)) % 9;
                    const C<R> u = ST == 1 ? Uq[st][2] : U[st][q1];
                    C<R> F;
                    if constexpr (ST == 0) {
                        C<R> dx = d2u<R>(nb[1], u, nb[2]);
                        if (plain) {
                            if (xface) dx = fv[st];   // fv[st] is row r of the face (set where xface)
                        } else if (has_face) {        // wave-uniform: only the edge strips select
                            if (xface) dx = fv[st];
                            asm volatile("" : "+v"(dx.x), "+v"(dx.y));   // keeps the branch
                        }
                        const C<R> alap = lap2a<R>(dx, D[st][q2], clane_prev<R>(dx), clane_next<R>(dx), D[st][q1],
                                                   D[st][q0], lc.A76, lc.A112);
                        F = rhs_a<R>(alap, u, Vq[kr], s);
                    } else if constexpr (ST == 2) {   // a/h^2 (D^x + D^y) from the unscaled differences
                        const C<R> dx = d2u<R>(nb[1], u, nb[2]);
                        F = rhs_a<R>(cscale<R>(aih2, cadd<R>(dx, D[st][q2])), u, Vq[kr], s);
                    } else {   // five-point differences along x (lanes) and y (the row queue)
                        const C<R> xm1 = nb[1], xp1 = nb[2];
                        C<R> xm2 = nb[0], xp2 = nb[3];
                        if (has_face) {   // fv[st]: the face value of row r next to lane x = 1 / nx - 1
                            if (x == 1) xm2 = ghost<R>(xm1, u, fv[st]);
                            if (x == nx - 1) xp2 = ghost<R>(xp1, u, fv[st]);
                        }
                        C<R> ym2 = Uq[st][0], yp2 = Uq[st][4];
                        if (!plain) {
                            if (r == 1) ym2 = ghost<R>(Uq[st][1], u, sdy[0][lane]);
                            if (r == ny - 1) yp2 = ghost<R>(Uq[st][3], u, sdy[1][lane]);
                        }
                        const C<R> lap = cadd<R>(d4nc<R>(xm2, xm1, u, xp1, xp2, i12h2),
                                                 d4nc<R>(ym2, Uq[st][1], u, Uq[st][3], yp2, i12h2));
                        F = rhs<R>(lap, u, Vq[kr], aR, s);
                    }
                    const R rowf = (plain || (r >= 1 && r < ny)) ? R(1) : R(0);   // wave-uniform
                    if (st == 0) {
                        Kq[kr] = F;
                        outv = cvt<R, M>(axpy_m<R, M>(P[kr], plain ? ckl[0] : ckl[0] * rowf, F));
                    } else if (st < 3) {
                        Kq[kr] = kacc<R>(Kq[kr], F);
                        outv = cvt<R, M>(axpy_m<R, M>(P[kr], plain ? ckl[st] : ckl[st] * rowf, F));
                    } else if (wlane && r >= ys && (plain || r < y1)) {
                        pout[r * px + x + ox] = axpy_m<R, M>(P[kr], ck[3], cadd<R>(Kq[kr], F));
                    }
                }
                in = outv;
                if (st < 3) {
                    ring[st + 1][q0][RP + lane] = in;
#pragma unroll
                    for (int i = 0; i < 4; ++i) nb[i] = nbn[i];
                }
            }
        }
    };
    static_assert(Q >= 2, "the first two groups are the warm-up");
    const int gp = min(Q, max(2, (ny - jb - 8) / 9 + 1));   // groups 2 .. gp-1 are plain
#pragma unroll 1
    for (int g = 0; g < 2; ++g) group(g, std::false_type{});
#pragma unroll 1
    for (int g = 2; g < gp; ++g) group(g, std::true_type{});
#pragma unroll 1
    for (int g = gp; g < Q; ++g) group(g, std::false_type{});
}

}  // namespace wave2d
}  // namespace nlse
