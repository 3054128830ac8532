// On-chip 1D 2SHOC-RK4 solver body (shared by the stand-alone 1D kernel and the
// batched persistent kernel).  One workgroup of BS threads holds a whole field of
// up to BS * NPT nodes: Psi^n, K_tot and V in registers of the owning thread
// (node i belongs to thread i % BS), the stage field and D in LDS.  See
// solve1d.hip for the per-stage phases.
#pragma once

#include "kernels.h"

namespace nlse {

template <typename R>
__device__ __forceinline__ C<R> lap1d(const C<R> *sD, int64_t i, R c76, R c112)
{
    return csub<R>(cscale<R>(c76, sD[i]), cscale<R>(c112, cadd<R>(sD[i + 1], sD[i - 1])));
}

// smem_raw: 2 (n + 1) stage-precision complex values of LDS.
template <typename R, typename M, int BS, int NPT>
__device__ void solve1d_onchip(const Solve1DArgs &A, unsigned char *smem_raw)
{
    const int64_t n = A.L.nx;                 // nodes 0..n
    C<R> *sin = (C<R> *)smem_raw;             // stage field
    C<R> *sD = sin + (n + 1);                 // step-1 array
    const int t = threadIdx.x;
    constexpr int BS1D = BS;
    const R a = (R)A.c.a, s = (R)A.c.s, ih2 = (R)A.c.ih2, c76 = (R)A.c.c76, c112 = (R)A.c.c112;
    const R ia = (R)A.c.ia, two = (R)2;
    const R k2 = (R)A.k2, kk = (R)A.k, k6 = (R)A.k6;
    const bool msd = A.msd != 0;
    C<M> *gpsi = (C<M> *)A.psin;
    const R *gV = (const R *)A.V;
    const int64_t o = A.L.ox;

    C<M> pn[NPT];
    C<R> kt[NPT], F[NPT];
    R vv[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int64_t i = t + (int64_t)j * BS1D;
        pn[j] = mk<M>(M(0), M(0));
        kt[j] = czero<R>();
        F[j] = czero<R>();
        vv[j] = R(0);
        if (i <= n) {
            pn[j] = gpsi[o + i];
            vv[j] = gV ? gV[o + i] : R(0);
            sin[i] = cvt<R, M>(pn[j]);
        }
    }
    auto Vat = [&](int64_t i) -> R { return gV ? gV[o + i] : R(0); };
    auto nonl = [&](int64_t i) -> R { const C<R> u = sin[i]; return s * (u.x * u.x + u.y * u.y) - Vat(i); };
    // second difference at an interior node straight from the stage field
    auto d2 = [&](int64_t i) -> C<R> {
        return cscale<R>(ih2, cadd<R>(csub<R>(sin[i + 1], cscale<R>(two, sin[i])), sin[i - 1]));
    };
    // F at an interior node from D in LDS
    auto Fat = [&](int64_t i) -> C<R> {
        const C<R> u = sin[i];
        const C<R> z = cadd<R>(cscale<R>(a, lap1d<R>(sD, i, c76, c112)), cscale<R>(nonl(i), u));
        return mk<R>(-z.y, z.x);
    };

    for (int64_t step = 0; step < A.nsteps; ++step) {
        for (int stage = 1; stage <= 4; ++stage) {
            __syncthreads();
            // phase A: step 1 with its boundary closure
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                const int64_t i = t + (int64_t)j * BS1D;
                if (i > n) continue;
                if (i > 0 && i < n) {
                    sD[i] = d2(i);
                } else {
                    const int64_t bm1 = (i == 0) ? 1 : n - 1;
                    const C<R> ub = sin[i];
                    if (!msd) {
                        sD[i] = cscale<R>(-nonl(i) * ia, ub);
                    } else {
                        const C<R> ui = sin[bm1], Di = d2(bm1);
                        const R den = ui.x * ui.x + ui.y * ui.y;
                        const R ratio = den != R(0) ? (Di.x * ui.x + Di.y * ui.y) / den : R(0);
                        sD[i] = cscale<R>(ratio + (nonl(bm1) - nonl(i)) * ia, ub);
                    }
                }
            }
            __syncthreads();
            // phase B: step 2 and F
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                const int64_t i = t + (int64_t)j * BS1D;
                F[j] = czero<R>();
                if (i > n) continue;
                if (i > 0 && i < n) {
                    F[j] = Fat(i);
                } else if (msd) {
                    const int64_t bm1 = (i == 0) ? 1 : n - 1;
                    const C<R> Fi = Fat(bm1), ui = sin[bm1], ub = sin[i];
                    const R den = ui.x * ui.x + ui.y * ui.y;
                    const R im = den != R(0) ? (Fi.y * ui.x - Fi.x * ui.y) / den : R(0);
                    F[j] = mk<R>(-im * ub.y, im * ub.x);
                }
            }
            __syncthreads();
            // phase C: RK4 array operations of this stage
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                const int64_t i = t + (int64_t)j * BS1D;
                if (i > n) continue;
                if ((i == 0 || i == n) && !msd) continue;   // Dirichlet nodes never change
                C<R> nxt;
                if (stage == 1) {
                    kt[j] = F[j];
                    const C<R> inc = cscale<R>(k2, F[j]);
                    nxt = cvt<R, M>(mk<M>(pn[j].x + (M)inc.x, pn[j].y + (M)inc.y));
                } else if (stage <= 3) {
                    kt[j] = cadd<R>(kt[j], cscale<R>(two, F[j]));
                    const C<R> inc = cscale<R>(stage == 2 ? k2 : kk, F[j]);
                    nxt = cvt<R, M>(mk<M>(pn[j].x + (M)inc.x, pn[j].y + (M)inc.y));
                } else {
                    const C<R> inc = cscale<R>(k6, cadd<R>(kt[j], F[j]));
                    pn[j] = mk<M>(pn[j].x + (M)inc.x, pn[j].y + (M)inc.y);
                    nxt = cvt<R, M>(pn[j]);
                }
                sin[i] = nxt;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int64_t i = t + (int64_t)j * BS1D;
        if (i <= n) gpsi[o + i] = pn[j];
    }
}

}  // namespace nlse
