// On-chip 1D 2SHOC-RK4 solver body (shared by the stand-alone 1D kernel and the
// batched persistent kernel).  One workgroup of BS threads holds a whole field
// of up to BS * NPT nodes and runs all requested RK4 steps; HBM is touched only
// to load Psi^n at the start and store it at the end.
//
// Layout.  Thread t owns npt consecutive nodes i = t*npt - sh + j, j < npt, with
// npt = max(3, ceil((n+1)/BS)) and a shift sh in {0, 1} chosen so that each
// boundary node shares its thread with its interior neighbour (node 0 is never
// a thread's last node, node n never a thread's first).  Psi^n (master type),
// K_tot, V, the stage field and D of the owned nodes live in registers.  Per
// stage (Sec. 2.1 Eqs. 2shoc1d-2shoc1d2, Sec. 3.1-3.2):
//   1. the end nodes of the stage field are exchanged with the neighbouring
//      threads: DPP lane shifts inside a wave, LDS across waves (barrier);
//   2. D = delta^2 Psi on the owned nodes; boundary D_b by the Dirichlet rule
//      (Eq. dbc_lap) or the MSD rule (Eq. msdbc_lap, from D_{b-1});
//   3. the end values of D are exchanged the same way (barrier);
//   4. Lap (Eq. 2shoc1d2) and F on interior nodes; boundary F_b: Dirichlet 0
//      (Eq. dbc_ut) or MSD i Im(F_{b-1}/Psi_{b-1}) Psi_b (Eq. msdbc_ut);
//   5. the RK4 array operations of the stage (Eq. RK4) on every node that moves.
// The alternative Laplacians (Dirichlet only) replace steps 2-4: CD takes D itself;
// the non-compact five-point stencil exchanges two end nodes per side in step 1
// and forms every slot's Laplacian before step 5 overwrites the slots it reads.
// Either keeps the second barrier of the stage.
#pragma once

#include "dpp.h"
#include "kernels.h"
#include "point.h"

namespace nlse {

// LDS the solver needs: the cross-wave exchange slots.
template <typename R, int BS>
constexpr size_t onchip1d_lds() { return sizeof(C<R>) * 2 * (BS / 64) * 2; }

// Largest field (nodes) the solver holds; the caller guarantees n + 1 <= this.
template <int BS, int NPT>
constexpr int64_t onchip1d_max_nodes() { return (int64_t)BS * NPT; }

// End values of the neighbouring threads of an array of npt owned slots: prev = last
// slot of thread t-1, next = first slot of thread t+1 (DPP inside the wave, the LDS
// slots `edge` [wave][first, last] across waves).  Contains a workgroup barrier.
template <typename R, int NPT, int NWV>
__device__ __forceinline__ void exchange1d(const C<R> (&v)[NPT], int npt, int lane, int wv, C<R> (*edge)[2],
                                           C<R> &prev, C<R> &next)
{
    C<R> last = v[0];
#pragma unroll
    for (int j = 1; j < NPT; ++j)
        if (j == npt - 1) last = v[j];
    const C<R> first = v[0];
    prev = clane_prev<R>(last);
    next = clane_next<R>(first);
    if (lane == 0) edge[wv][0] = first;
    if (lane == 63) edge[wv][1] = last;
    __syncthreads();
    if (lane == 0 && wv > 0) prev = edge[wv - 1][1];
    if (lane == 63 && wv < NWV - 1) next = edge[wv + 1][0];
}

// As exchange1d, with the two end values on each side: p1, p2 = last and second-to-last
// slot of thread t-1, n1, n2 = first and second slot of thread t+1 (npt >= 3).
template <typename R, int NPT, int NWV>
__device__ __forceinline__ void exchange1d2(const C<R> (&v)[NPT], int npt, int lane, int wv, C<R> (*edge)[4],
                                            C<R> &p1, C<R> &p2, C<R> &n1, C<R> &n2)
{
    C<R> last = v[0], last2 = v[0];
#pragma unroll
    for (int j = 1; j < NPT; ++j) {
        if (j == npt - 1) last = v[j];
        if (j == npt - 2) last2 = v[j];
    }
    const C<R> first = v[0], second = v[1];
    p1 = clane_prev<R>(last);
    p2 = clane_prev<R>(last2);
    n1 = clane_next<R>(first);
    n2 = clane_next<R>(second);
    if (lane == 0) {
        edge[wv][0] = first;
        edge[wv][1] = second;
    }
    if (lane == 63) {
        edge[wv][2] = last2;
        edge[wv][3] = last;
    }
    __syncthreads();
    if (lane == 0 && wv > 0) {
        p1 = edge[wv - 1][3];
        p2 = edge[wv - 1][2];
    }
    if (lane == 63 && wv < NWV - 1) {
        n1 = edge[wv + 1][0];
        n2 = edge[wv + 1][1];
    }
}

// ST selects the Laplacian: 0 2SHOC, 1 the non-compact five-point stencil (beyond a boundary
// node b the ghost 2 Psi_b - Psi_{b-+1} + h^2 D_b, D_b of Eq. dbc_lap), 2 the second-order CD; the alternatives with Dirichlet
// boundaries only.  Every path takes exactly two workgroup barriers per stage (the idle
// waves below count on it).
template <typename R, typename M, int BS, int NPT, int ST = 0>
__device__ void solve1d_onchip(const Solve1DArgs &A, unsigned char *smem_raw)
{
    static_assert(BS % 64 == 0 && NPT >= 3, "whole waves, at least three nodes per thread");
    constexpr int NWV = BS / 64;
    C<R>(*edge)[NWV][2] = reinterpret_cast<C<R>(*)[NWV][2]>(smem_raw);   // [exchange][wave][first, last]
    C<R>(*edge4)[4] = reinterpret_cast<C<R>(*)[4]>(smem_raw);           // [wave][two first, two last] (ST 1)
    const int n = __builtin_amdgcn_readfirstlane((int)A.L.nx);   // nodes 0..n
    const int npt = max(3, (n + 1 + BS - 1) / BS);
    const int sh = (n % npt == 0) ? 1 : 0;   // BS * npt >= n + 1 + sh holds (see the layout note)
    const int t = threadIdx.x, lane = t & 63;
    const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int i0 = t * npt - sh;             // node of slot 0
    const int tn = (n + sh) / npt, jn = (n + sh) % npt;   // owner and slot of node n (jn >= 1)
    const bool msd = __builtin_amdgcn_readfirstlane(A.msd) != 0;

    const R a = (R)A.c.a, s = (R)A.c.s, ih2 = (R)A.c.ih2, c76 = (R)A.c.c76, c112 = (R)A.c.c112;
    const R ia = (R)A.c.ia;
    const R i12h2 = (R)(A.c.ih2 / 12.0), h2 = (R)(1.0 / A.c.ih2);
    const R k2 = (R)A.k2, kk = (R)A.k, k6 = (R)A.k6;
    C<M> *gpsi = (C<M> *)A.psin;
    const R *gV = (const R *)A.V;
    const int o = (int)A.L.ox;

    C<M> P[NPT];
    C<R> U[NPT], K[NPT], D[NPT];   // stage field, K_tot, step-1 values
    R Vv[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int i = i0 + j;
        const bool ok = j < npt && i >= 0 && i <= n;
        P[j] = ok ? gpsi[o + i] : mk<M>(M(0), M(0));
        Vv[j] = (ok && gV) ? gV[o + i] : R(0);
        U[j] = cvt<R, M>(P[j]);
        K[j] = czero<R>();
        D[j] = czero<R>();
    }

    // A wave whose first node lies beyond n owns no node: it only takes part in the two
    // barriers of every stage (s_barrier counts waves, not code locations).
    const bool busy = wv * 64 * npt - sh <= n;
    if (!busy) {
        for (int64_t b = 0; b < 8 * A.nsteps; ++b) __syncthreads();
        return;
    }
    for (int64_t step = 0; step < A.nsteps; ++step) {
#pragma unroll 1
        for (int st = 0; st < 4; ++st) {
            C<R> up, un, up2 = czero<R>(), un2 = czero<R>();
            if constexpr (ST == 1) {
                exchange1d2<R, NPT, NWV>(U, npt, lane, wv, edge4, up, up2, un, un2);
            } else {
                exchange1d<R, NPT, NWV>(U, npt, lane, wv, edge[0], up, un);
            }
            C<R> Fb = czero<R>();
            C<R> dp = czero<R>(), dn = czero<R>();
            // F at an interior slot (D and its neighbours dp, dn are set below before any call)
            auto Fint = [&](int j) {
                if constexpr (ST == 0) {
                    const C<R> dl = j == 0 ? dp : D[j > 0 ? j - 1 : 0];
                    const C<R> dr = j == npt - 1 ? dn : D[j + 1 < NPT ? j + 1 : j];
                    return rhs<R>(lap1<R>(D[j], dl, dr, c76, c112), U[j], Vv[j], a, s);
                } else {   // the Laplacian sits in D (formed before any slot of this stage moved)
                    return rhs<R>(D[j], U[j], Vv[j], a, s);
                }
            };
            if constexpr (ST == 0) {
                // step 1 on every owned slot (boundary and out-of-range slots are fixed below or unused)
#pragma unroll
                for (int j = 0; j < NPT; ++j) {
                    if (j >= npt) continue;
                    const C<R> lo = j == 0 ? up : U[j > 0 ? j - 1 : 0];
                    const C<R> hi = j == npt - 1 ? un : U[j + 1 < NPT ? j + 1 : j];
                    D[j] = d2<R>(lo, U[j], hi, ih2);
                }
                // boundary D_b: node 0 is slot sh of thread 0, node n slot jn of thread tn
#pragma unroll
                for (int j = 0; j < NPT; ++j) {
                    const bool b0 = t == 0 && j == sh, bn = t == tn && j == jn;
                    if (!(b0 || bn) || j >= npt) continue;
                    // interior neighbour: slot j + 1 for node 0, j - 1 for node n (static indices)
                    const int jp = j + 1 < NPT ? j + 1 : j, jq = j > 0 ? j - 1 : 0;   // constants once unrolled
                    const C<R> ub = U[j];
                    if (!msd) {
                        D[j] = cscale<R>(-nonlin<R>(ub, Vv[j], s) * ia, ub);
                    } else {
                        const C<R> ui = b0 ? U[jp] : U[jq], Di = b0 ? D[jp] : D[jq];
                        const R vi = b0 ? Vv[jp] : Vv[jq];
                        const R ratio = re_div<R>(Di, ui);
                        D[j] = cscale<R>(ratio + (nonlin<R>(ui, vi, s) - nonlin<R>(ub, Vv[j], s)) * ia, ub);
                    }
                }
                exchange1d<R, NPT, NWV>(D, npt, lane, wv, edge[1], dp, dn);
                // MSD boundary F_b, from F_{b-1} of the unchanged stage field (before any update)
                if (msd) {
#pragma unroll
                    for (int j = 0; j < NPT; ++j) {
                        const bool b0 = t == 0 && j == sh, bn = t == tn && j == jn;
                        if (!(b0 || bn) || j >= npt) continue;
                        const int jp = j + 1 < NPT ? j + 1 : j, jq = j > 0 ? j - 1 : 0;   // constants once unrolled
                        const C<R> Fi = b0 ? Fint(jp) : Fint(jq), ui = b0 ? U[jp] : U[jq], ub = U[j];
                        const R im = im_div<R>(Fi, ui);
                        Fb = mk<R>(-im * ub.y, im * ub.x);
                    }
                }
            } else if constexpr (ST == 2) {   // CD: the step-1 value is the Laplacian
#pragma unroll
                for (int j = 0; j < NPT; ++j) {
                    if (j >= npt) continue;
                    const C<R> lo = j == 0 ? up : U[j > 0 ? j - 1 : 0];
                    const C<R> hi = j == npt - 1 ? un : U[j + 1 < NPT ? j + 1 : j];
                    D[j] = d2<R>(lo, U[j], hi, ih2);
                }
                __syncthreads();
            } else {   // (-Psi_{+2} + 16 Psi_{+1} - 30 Psi + 16 Psi_{-1} - Psi_{-2}) / (12 h^2)
#pragma unroll
                for (int j = 0; j < NPT; ++j) {
                    if (j >= npt) continue;
                    const int i = i0 + j;
                    const C<R> u = U[j];
                    const C<R> m1 = j >= 1 ? U[j > 0 ? j - 1 : 0] : up;
                    const C<R> q1 = j + 1 < npt ? U[j + 1 < NPT ? j + 1 : j] : un;
                    C<R> m2 = j >= 2 ? U[j > 1 ? j - 2 : 0] : (j == 1 ? up : up2);
                    C<R> q2 = j + 2 < npt ? U[j + 2 < NPT ? j + 2 : j] : (j + 1 < npt ? un : un2);
                    // beyond node 0 or n the ghost carries h^2 D_b of Eq. dbc_lap; the boundary
                    // node is the neighbouring slot of the same thread (slot j-1 for node 0,
                    // j+1 for node n)
                    if (i == 1) {         // m1 is Psi_0
                        const R vb = Vv[j > 0 ? j - 1 : 0];
                        m2 = ghost<R>(m1, u, cscale<R>(-nonlin<R>(m1, vb, s) * ia * h2, m1));
                    }
                    if (i == n - 1) {     // q1 is Psi_n
                        const R vb = Vv[j + 1 < NPT ? j + 1 : j];
                        q2 = ghost<R>(q1, u, cscale<R>(-nonlin<R>(q1, vb, s) * ia * h2, q1));
                    }
                    D[j] = d4nc<R>(m2, m1, u, q1, q2, i12h2);
                }
                __syncthreads();
            }
            // F and the RK4 array operations of this stage; a slot's update touches only its
            // own stage value, which no other slot reads any more.  Dirichlet boundary nodes
            // and slots outside 0..n never change.
            const R ckst = st == 0 ? k2 : st == 1 ? k2 : st == 2 ? kk : k6;
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                const int i = i0 + j;
                if (j >= npt || i < 0 || i > n) continue;
                const bool bnd = i == 0 || i == n;
                if (!msd && bnd) continue;
                const C<R> F = bnd ? Fb : Fint(j);
                if (st == 0) {
                    K[j] = F;
                    U[j] = cvt<R, M>(axpy_m<R, M>(P[j], ckst, F));
                } else if (st < 3) {
                    K[j] = kacc<R>(K[j], F);
                    U[j] = cvt<R, M>(axpy_m<R, M>(P[j], ckst, F));
                } else {
                    P[j] = axpy_m<R, M>(P[j], ckst, cadd<R>(K[j], F));
                    U[j] = cvt<R, M>(P[j]);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const int i = i0 + j;
        if (j < npt && i >= 0 && i <= n) gpsi[o + i] = P[j];
    }
}

}  // namespace nlse
