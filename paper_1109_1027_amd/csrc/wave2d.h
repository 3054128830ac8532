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
// the same for segments of ng <= Q row groups (9 ng - 2 HALO rows)
__host__ __device__ inline int segments_ng(int64_t ny, int ng)
{
    const int sr = 9 * ng - 2 * HALO;
    return (int)((ny - 1 + sr - 1) / sr);
}

// Under MSD: whether the window of segment `seg` (ng row groups) meets a face row, i.e. starts
// above row 0 or reaches input row ny + 1, where the closures of rows 0 and ny act (the window
// placement is that of step2d_wave).
__host__ __device__ inline bool meets_face_rows(int ny, int seg, int ng)
{
    const int sr = 9 * ng - 2 * HALO, yend = ny + 1;
    const int ys = 1 + sr * seg;
    const int y0 = seg == segments_ng(yend, ng) - 1 ? (yend - sr > 1 ? yend - sr : 1) : ys;
    const int jb = y0 - HALO;
    return jb < 0 || jb + 9 * ng >= ny;
}

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

// MSD face value (Sec. 3.2, Eq. msdbc_lap) at a face node b in 2D, in the unscaled form the stages
// read (h^2 D^a_b), from unscaled second differences: dqx and dqy at q = b-1 along x and y, dbt at b
// along the face.  The operations and their order are those of the MSD boundary kernel.
template <typename R>
__device__ __forceinline__ C<R> msd_face(C<R> ub, C<R> uq, R vb, R vq, C<R> dqx, C<R> dqy, C<R> dbt, R ih2, R h2,
                                         R s, R ia)
{
#pragma clang fp contract(off)
    const C<R> Dq = cadd<R>(cadd<R>(czero<R>(), mk<R>(dqx.x * ih2, dqx.y * ih2)), mk<R>(dqy.x * ih2, dqy.y * ih2));
    const R fac = re_div<R>(Dq, uq) + (nonlin<R>(uq, vq, s) - nonlin<R>(ub, vb, s)) * ia;
    const C<R> Db = csub<R>(mk<R>(fac * ub.x, fac * ub.y), mk<R>(dbt.x * ih2, dbt.y * ih2));
    return unscaled<R>(Db, h2);
}

// strip < strips(nx) and seg < segments_ng(ny + MSD, ng), 2 <= ng <= Q row groups per segment, all
// wave-uniform; the field has < 2^31 elements.
//
// MSD: the boundary nodes evolve.  The face values come from the MSD closure of each stage's input
// on the spot, and F_b from F at b-1 (the diagonal interior node at a corner):
//   faces x = 0, nx (edge lanes of the edge strips): everything is in the row being processed; the
//     closure is formed at b-1 (x = 1, nx-1), which uses it as its D^x neighbour, and the edge
//     lane takes Im(F/Psi) from there;
//   face y = 0: the closure of row 0 needs D^y at row 1 and is formed one row later than a face
//     value would be read (before its first use); F_b of row 0 needs F of row 1, so each stage
//     hands row 0 of its output to the next stage one row late, straight into that stage's rings
//     (it is first read the row after);
//   face y = ny: F_b of row ny is formed with F of row ny-1, one row before row ny's output, and
//     kept in LDS meanwhile.
// The segments cover rows 1 .. ny (row ny is stored by the last one) and row 0 by the first.
// ST selects the Laplacian as in the stage kernels: 0 the per-axis 2SHOC form, 1 the
// non-compact five-point stencil (ghosts 2 Psi_b - Psi_{b-+1} + h^2 D^a_b beyond a face), 2 the
// second-order CD.
// EDGE = false: the caller guarantees that the wave's 64 columns hold no face column (x = 0, nx),
// and the face code is compiled out (under MSD it is long, and the instruction cache is shared).
// YF = false (MSD): the caller guarantees that the task's window meets neither face row
// (meets_face_rows), and the closures of rows 0 and ny are compiled out as well: they are long, and
// every checked row group would carry them although only the first and last segments use them.
template <typename R, typename M, int Q, int PD = 1, int ST = 0, bool MSD = false, bool EDGE = true, bool YF = true>
__device__ __forceinline__ void step2d_wave(const Step2DArgs &A, int strip, int seg, int lane, Staging<R, Q> &S,
                                            int ng = Q)
{
    static_assert(!MSD || ST == 0, "MSD with the per-axis 2SHOC form");
    auto &sdx = S.sdx;
    auto &sdy = S.sdy;
    auto &ring = S.ring;
    const int SEG = 9 * ng - 2 * HALO;      // output rows per segment
    constexpr int FR = face_rows<Q>();
    lds_order();        // earlier reads of the staging come first
    const int nx = (int)A.L.nx, ny = (int)A.L.ny, px = (int)A.L.px, ox = (int)A.L.ox;
    const int xs = 1 + SW * strip - HALO;   // column of lane 0
    const int x = xs + lane;
    const bool xin = x >= 0 && x <= nx;
    const bool xint = x >= 1 && x < nx;
    const bool xface = x == 0 || x == nx;
    // lanes that store Psi^{n+1}: the middle 48; under MSD also a face column (x = 0 at lane
    // HALO-1 of the first strip, x = nx at most at lane HALO+SW of the last)
    const bool wlane = (xint && lane >= HALO && lane < HALO + SW) ||
                       (MSD && xface && lane >= HALO - 1 && lane <= HALO + SW);
    const bool has_lo = EDGE && xs <= 0, has_hi = EDGE && xs + 63 >= nx;   // the faces x = 0 / nx in this strip
    const bool has_face = has_lo || has_hi;                 // wave-uniform
    // The task stores rows ys .. y1-1.  Its window of rows starts at y0 = ys, except in the last
    // segment, whose window ends at the face (y0 = ny - SEG, overlapping the segment before it):
    // then the face rows meet the pipeline only in the last group.
    const int yend = MSD ? ny + 1 : ny;     // rows 1 .. yend-1 are stored by the segments
    const int ys = 1 + SEG * seg, y1 = min(ys + SEG, yend);
    const int y0 = seg == segments_ng(yend, ng) - 1 ? max(1, yend - SEG) : ys;
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
    for (int i = 0; i < 3; ++i) ckl[i] = (MSD ? xin : xint) ? ck[i] : R(0);
    const C<M> *__restrict__ pin = (const C<M> *)A.psi_in;
    C<M> *__restrict__ pout = (C<M> *)A.psi_out;
    const R *__restrict__ V = (const R *)A.V;
    const C<R> *__restrict__ DBx = (const C<R> *)A.DB[0];
    const C<R> *__restrict__ DBy = (const C<R> *)A.DB[1];

    // MSD reuses sdy: [0] F_b of row ny until its output row, [1] row 0 of a stage's input
    if (!MSD) sdy[0][lane] = xin ? unscaled<R>(dev_ld(DBy + x), lc.h2) : czero<R>();   // unscaled, like d2u
    if (!MSD) sdy[1][lane] = xin ? unscaled<R>(dev_ld(DBy + nx + 1 + x), lc.h2) : czero<R>();
    const R ih2 = (R)A.c.ih2, ia = (R)A.c.ia;
    if (!MSD && has_face) {
        for (int i = lane; i < FR; i += 64) {
            const int r = jb - HALO + i;
            const bool ok = r >= 0 && r <= ny;
            sdx[0][i] = ok ? unscaled<R>(dev_ld(DBx + r), lc.h2) : czero<R>();
            sdx[1][i] = ok ? unscaled<R>(dev_ld(DBx + ny + 1 + r), lc.h2) : czero<R>();
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
        pv = dev_ld(pin + o);
        vv = dev_ld(V + o);
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
    auto group = [&](const int g, auto plain_t, auto yf_t) __attribute__((always_inline)) {   // inlined: the rings stay in registers
        constexpr bool plain = decltype(plain_t)::value;
        constexpr bool yf = decltype(yf_t)::value;
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
            if (!MSD && has_face) {
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
                        if constexpr (!MSD) {
                            if (m - 1 == 0) dy = sdy[0][lane];
                            if (m - 1 == ny) dy = sdy[1][lane];
                        } else if (yf && m - 1 == ny) {   // closure of face row ny: b = row ny, q = row ny-1
                            const int kq = (p + 18 - 2 * (st + 1)) % 9;   // ring slot of row m-2
                            const C<R> *rb = ring[st][q2] + RP + lane;     // row ny (m-1)
                            const C<R> dbt = d2u<R>(rb[-1], U[st][q2], rb[1]);
                            const C<R> dqx = d2u<R>(nb[1], U[st][q1], nb[2]);
                            dy = msd_face<R>(U[st][q2], U[st][q1], Vq[(kq + 1) % 9], Vq[kq], dqx, D[st][q2], dbt, ih2,
                                             lc.h2, s, ia);
                        }
                    }
                    D[st][q0] = dy;
                    if constexpr (MSD) {
                        if (yf && !plain && jb < 0 && m == 2) {   // closure of face row 0 (b = row 0, q = row 1)
                            const int kq = (p + 18 - 2 * (st + 1)) % 9;   // ring slot of row 0 (m-2)
                            const C<R> *rq = ring[st][q2] + RP + lane;     // row 1 (m-1)
                            const C<R> dqx = d2u<R>(rq[-1], U[st][q2], rq[1]);
                            const C<R> dbt = d2u<R>(nb[1], U[st][q1], nb[2]);
                            D[st][q2] = msd_face<R>(U[st][q1], U[st][q2], Vq[kq], Vq[(kq + 1) % 9], dqx, dy, dbt, ih2,
                                                    lc.h2, s, ia);
                        }
                    }
                }
                C<R> outv = czero<R>();
                if (plain || t >= 4 * (st + 1)) {    // earlier output rows feed nothing
                    const int r = m - 2;    // output row
                    const int kr = (p + 18 - 2 * (st + 1)) % 9;
                    const C<R> u = ST == 1 ? Uq[st][2] : U[st][q1];
                    C<R> F;
                    // MSD: Im(F/Psi) at b-1 for every lane (this lane's; the neighbour's on an edge lane,
                    // whose own F is not read), formed only where a boundary node needs it
                    auto w_bm1 = [&](const C<R> &Fv) {
                        R w = im_div<R>(Fv, u);
                        if (has_lo) {
                            const R wn = lane_next(w);
                            if (x == 0) w = wn;
                        }
                        if (has_hi) {
                            const R wp = lane_prev(w);
                            if (x == nx) w = wp;
                        }
                        return w;
                    };
                    if constexpr (ST == 0) {
                        C<R> dx = d2u<R>(nb[1], u, nb[2]);
                        C<R> dxl, dxr;
                        if constexpr (MSD) {
                            dxl = clane_prev<R>(dx);
                            dxr = clane_next<R>(dx);
                            // closures of the faces x = 0 and x = nx, formed at b-1 (only the faces
                            // the strip holds: the whole wave pays for the one lane)
                            if (has_lo) {
                                const R vp = lane_prev(Vq[kr]);
                                const C<R> dyp = clane_prev<R>(D[st][q2]);
                                if (x == 1)
                                    dxl = msd_face<R>(nb[1], u, vp, Vq[kr], dx, D[st][q2], dyp, ih2, lc.h2, s, ia);
                            }
                            if (has_hi) {
                                const R vn = lane_next(Vq[kr]);
                                const C<R> dyn = clane_next<R>(D[st][q2]);
                                if (x == nx - 1)
                                    dxr = msd_face<R>(nb[2], u, vn, Vq[kr], dx, D[st][q2], dyn, ih2, lc.h2, s, ia);
                            }
                        } else {
                            if (plain) {
                                if (xface) dx = fv[st];   // fv[st] is row r of the face (set where xface)
                            } else if (has_face) {        // wave-uniform: only the edge strips select
                                if (xface) dx = fv[st];
                                asm volatile("" : "+v"(dx.x), "+v"(dx.y));   // keeps the branch
                            }
                            dxl = clane_prev<R>(dx);
                            dxr = clane_next<R>(dx);
                        }
                        const C<R> alap = lap2a<R>(dx, D[st][q2], dxl, dxr, D[st][q1], D[st][q0], lc.A76, lc.A112);
                        F = rhs_a<R>(alap, u, Vq[kr], s);
                        if constexpr (MSD) {
                            if (has_face) {   // F_b on the edge lanes (Eq. msdbc_ut)
                                const R w = w_bm1(F);
                                if (xface) F = msd_fb<R>(w, u);
                            }
                        }
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
                    if constexpr (MSD && yf) {
                        if (!plain) {
                            if (m == ny + 1) {   // F_b of row ny (b-1 = row ny-1, this row), kept in LDS
                                sdy[0][lane] = msd_fb<R>(w_bm1(F), U[st][q2]);
                            } else if (r == ny) {
                                F = sdy[0][lane];
                            }
                            if (jb < 0 && m == 3) {   // row 0 of this stage's output, one row late
                                const int k0 = (kr + 8) % 9;   // ring slot of row 0 (r - 1)
                                // (assignments, not a select of addresses, keep the rings in registers)
                                C<M> p0;
                                if (st == 3) p0 = dev_ld(pin + xc + ox);   // stage 4: row 0's ring slot is reused by now
                                else p0 = P[k0];
                                C<R> ub;
                                if (st == 0) ub = cvt<R, M>(P[k0]);
                                else ub = sdy[1][lane];
                                const C<R> Fb = msd_fb<R>(w_bm1(F), ub);
                                if (st == 0) {
                                    Kq[k0] = Fb;
                                } else if (st < 3) {
                                    Kq[k0] = kacc<R>(Kq[k0], Fb);
                                } else if (wlane && ys == 1) {
                                    dev_st(pout + x + ox, axpy_m<R, M>(p0, ck[3], cadd<R>(Kq[k0], Fb)));
                                }
                                if (st < 3) {   // into the next stage's rings, where row 0 is row m'-1
                                    const C<R> o0 = cvt<R, M>(axpy_m<R, M>(p0, ckl[st], Fb));
                                    U[st + 1][q2] = o0;
                                    ring[st + 1][q2][RP + lane] = o0;
                                    sdy[1][lane] = o0;
                                }
                            }
                        }
                    }
                    // rows outside 1 .. ny-1 (Dirichlet) or 1 .. ny (MSD) keep Psi^n; under MSD their
                    // K_tot slots are left alone (row 0's is filled one row late)
                    const bool rin = plain || (r >= 1 && (MSD ? r <= ny : r < ny));   // wave-uniform
                    const R rowf = rin ? R(1) : R(0);
                    if (st == 0) {
                        if (!MSD || rin) Kq[kr] = F;
                        outv = cvt<R, M>(axpy_m<R, M>(P[kr], plain ? ckl[0] : ckl[0] * rowf, F));
                    } else if (st < 3) {
                        if (!MSD || rin) Kq[kr] = kacc<R>(Kq[kr], F);
                        outv = cvt<R, M>(axpy_m<R, M>(P[kr], plain ? ckl[st] : ckl[st] * rowf, F));
                    } else if (wlane && r >= ys && (plain || r < y1)) {
                        dev_st(pout + r * px + x + ox, axpy_m<R, M>(P[kr], ck[3], cadd<R>(Kq[kr], F)));
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
    // groups 2 .. gp-1 are plain: the newest row of stage 1 stays below the face (MSD: one row more)
    const int gp = min(ng, max(2, (ny - jb - 8 - (MSD ? 1 : 0)) / 9 + 1));
    constexpr auto yf = std::integral_constant<bool, YF>{};
#pragma unroll 1
    for (int g = 0; g < 2; ++g) group(g, std::false_type{}, yf);
#pragma unroll 1
    for (int g = 2; g < gp; ++g) group(g, std::true_type{}, yf);
#pragma unroll 1
    for (int g = gp; g < ng; ++g) group(g, std::false_type{}, yf);
}

}  // namespace wave2d
}  // namespace nlse
