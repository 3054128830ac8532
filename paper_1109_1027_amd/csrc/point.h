// Point-wise pieces of one 2SHOC-RK4 stage, shared by every 2D kernel.  Every
// fused multiply-add is written out and automatic contraction is off, so all
// kernels that use these helpers perform the same roundings in the same order:
// their results are bit-identical, whatever the tiling or the fusion of stages.
#pragma once

#include "common.h"

namespace nlse {

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Step 1 along one axis: delta^2 Psi = (Psi_{+1} - 2 Psi_0 + Psi_{-1}) / h^2
// (Sec. 2.1, Eq. 2shoc1d: the second-order central difference).  2 Psi_0 is
// exact, so the fma rounds Psi_{+1} - 2 Psi_0 once, as the plain expression does.
template <typename R>
__device__ __forceinline__ C<R> d2(C<R> lo, C<R> c, C<R> hi, R ih2)
{
#pragma clang fp contract(off)
    return mk<R>((fmar(R(-2), c.x, hi.x) + lo.x) * ih2, (fmar(R(-2), c.y, hi.y) + lo.y) * ih2);
}

// Step 1 along one axis without the 1/h^2 factor, (Psi_{+1} - 2 Psi_0) + Psi_{-1}: the 2D
// kernels move 1/h^2 (and a) into the step-2 coefficients (lap2a), two multiplications
// fewer per difference.
template <typename R>
__device__ __forceinline__ C<R> d2u(C<R> lo, C<R> c, C<R> hi)
{
#pragma clang fp contract(off)
    return mk<R>(fmar(R(-2), c.x, hi.x) + lo.x, fmar(R(-2), c.y, hi.y) + lo.y);
}

// Step 2 of the per-axis 2D form (Sec. 2.2, Eqs. 2d2shocMs1-2): sum over both axes of
// D^a - (1/12) delta_a^2 D^a, written as (7/6)(D^x + D^y) - (1/12)(neighbour sums).
template <typename R>
__device__ __forceinline__ C<R> lap2(C<R> dx, C<R> dy, C<R> dxl, C<R> dxr, C<R> dyd, C<R> dyu, R c76, R c112)
{
#pragma clang fp contract(off)
    const R ax = dx.x + dy.x, ay = dx.y + dy.y;
    const R bx = (dxr.x + dxl.x) + (dyu.x + dyd.x), by = (dxr.y + dxl.y) + (dyu.y + dyd.y);
    return mk<R>(fmar(c76, ax, -(c112 * bx)), fmar(c76, ay, -(c112 * by)));
}

// Step 2 of the per-axis 3D form (Sec. 2.3, Eqs. 3d2shocMs1-2): (7/6)(D^x + D^y + D^z)
// - (1/12)(sum of the six axis neighbours' D^a).
template <typename R>
__device__ __forceinline__ C<R> lap3(C<R> dx, C<R> dy, C<R> dz, C<R> dxl, C<R> dxr, C<R> dyd, C<R> dyu,
                                     C<R> dzm, C<R> dzp, R c76, R c112)
{
#pragma clang fp contract(off)
    const R ax = (dx.x + dy.x) + dz.x, ay = (dx.y + dy.y) + dz.y;
    const R bx = ((dxr.x + dxl.x) + (dyu.x + dyd.x)) + (dzp.x + dzm.x);
    const R by = ((dxr.y + dxl.y) + (dyu.y + dyd.y)) + (dzp.y + dzm.y);
    return mk<R>(fmar(c76, ax, -(c112 * bx)), fmar(c76, ay, -(c112 * by)));
}

// a Lap of the per-axis 2D form from unscaled second differences (d2u):
// A76 = a (7/6) / h^2, A112 = a (1/12) / h^2; otherwise as lap2.
template <typename R>
__device__ __forceinline__ C<R> lap2a(C<R> dx, C<R> dy, C<R> dxl, C<R> dxr, C<R> dyd, C<R> dyu, R A76, R A112)
{
    return lap2<R>(dx, dy, dxl, dxr, dyd, dyu, A76, A112);
}

// Non-compact fourth-order second difference along one axis (Sec. 2.1, the stencil the
// 2SHOC scheme is compared with): (-Psi_{+2} + 16 Psi_{+1} - 30 Psi_0 + 16 Psi_{-1} - Psi_{-2})
// / (12 h^2), accumulated left to right; i12h2 = 1 / (12 h^2).
template <typename R>
__device__ __forceinline__ C<R> d4nc(C<R> m2, C<R> m1, C<R> c, C<R> p1, C<R> p2, R i12h2)
{
#pragma clang fp contract(off)
    const R tx = fmar(R(16), m1.x, fmar(R(-30), c.x, fmar(R(16), p1.x, -p2.x))) - m2.x;
    const R ty = fmar(R(16), m1.y, fmar(R(-30), c.y, fmar(R(16), p1.y, -p2.y))) - m2.y;
    return mk<R>(tx * i12h2, ty * i12h2);
}

// Ghost value one node beyond a Dirichlet boundary node b for the non-compact stencil:
// 2 Psi_b - Psi_{b-+1} + h^2 D^a_b (h2db = h^2 D^a_b), the value whose second difference at b
// is the step-1 face value D^a_b of Eq. dbc_lap.  With it the five-point stencil next to the
// boundary equals the 2SHOC combination there (Sec. 2.1); with zero boundary values it is
// the odd reflection 2 Psi_b - Psi_{b-+1}.
template <typename R>
__device__ __forceinline__ C<R> ghost(C<R> b, C<R> inner, C<R> h2db)
{
#pragma clang fp contract(off)
    return mk<R>(fmar(R(2), b.x, -inner.x) + h2db.x, fmar(R(2), b.y, -inner.y) + h2db.y);
}

// Step 2 of the 1D form (Sec. 2.1, Eq. 2shoc1d2): (7/6) D_i - (1/12)(D_{i+1} + D_{i-1}).
template <typename R>
__device__ __forceinline__ C<R> lap1(C<R> d, C<R> dl, C<R> dr, R c76, R c112)
{
#pragma clang fp contract(off)
    return mk<R>(fmar(c76, d.x, -(c112 * (dr.x + dl.x))), fmar(c76, d.y, -(c112 * (dr.y + dl.y))));
}

// The nonlinear-minus-potential factor s |Psi|^2 - V of Eq. NLSE.
template <typename R>
__device__ __forceinline__ R nonlin(C<R> u, R v, R s)
{
#pragma clang fp contract(off)
    return fmar(s, fmar(u.x, u.x, u.y * u.y), -v);
}

// Right-hand side of the NLSE (Sec. 1, Eq. NLSE) written as Psi_t = F:
// F = i [a Lap + (s |Psi|^2 - V) Psi].
template <typename R>
__device__ __forceinline__ C<R> rhs(C<R> lap, C<R> u, R v, R a, R s)
{
#pragma clang fp contract(off)
    const R nl = nonlin<R>(u, v, s);
    const R zx = fmar(nl, u.x, a * lap.x), zy = fmar(nl, u.y, a * lap.y);
    return mk<R>(-zy, zx);
}

// Dirichlet closure of step 1 on a boundary node (Sec. 3.2, Eq. dbc_lap):
// Lap_b = -(s |Psi_b|^2 - V_b) Psi_b / a, with ia = 1/a.  The per-axis kernels read
// D^a_b = Lap_b - (second differences along the face) on a face node normal to a;
// every kernel forms that value with these helpers in the master precision.
template <typename M>
__device__ __forceinline__ C<M> dirichlet_lapb(C<M> u, M v, M s, M ia)
{
#pragma clang fp contract(off)
    const M f = -(nonlin<M>(u, v, s) * ia);
    return mk<M>(f * u.x, f * u.y);
}

// F from a Lap (lap2a): F = i [a Lap + (s |Psi|^2 - V) Psi].
template <typename R>
__device__ __forceinline__ C<R> rhs_a(C<R> alap, C<R> u, R v, R s)
{
#pragma clang fp contract(off)
    const R nl = nonlin<R>(u, v, s);
    return mk<R>(-fmar(nl, u.y, alap.y), fmar(nl, u.x, alap.x));
}

// The step-2 coefficients of the 2D and 3D kernels and the factor h^2 that turns a face value D^a_b
// (scaled like a second derivative) into the unscaled form of d2u.
template <typename R>
struct Step2Coef {
    R A76, A112, h2;
};
template <typename R>
__host__ __device__ inline Step2Coef<R> step2_coef(double a, double c76, double c112, double ih2)
{
    return Step2Coef<R>{(R)(a * c76 * ih2), (R)(a * c112 * ih2), (R)(1.0 / ih2)};
}
template <typename R>
__device__ __forceinline__ C<R> unscaled(C<R> d, R h2)
{
    return mk<R>(d.x * h2, d.y * h2);
}

// Re(D / u) and Im(F / u) for the MSD closure (Sec. 3.2, Eqs. msdbc_lap, msdbc_ut), 0 when
// u = 0 (the ratio term is then dropped).  Numerator and u are first scaled by 2^-e with
// max(|u.x|, |u.y|) = f 2^e, 1/2 <= f < 1 (exact), so |u|^2 neither underflows nor loses its
// low bits when |u| is tiny (in FP32 |u|^2 is subnormal below |u| ~ 1e-19).
__device__ __forceinline__ float scale2(float v, int e) { return ldexpf(v, e); }
__device__ __forceinline__ double scale2(double v, int e) { return ldexp(v, e); }
__device__ __forceinline__ int exponent_of(float v) { int e; (void)frexpf(v, &e); return e; }
__device__ __forceinline__ int exponent_of(double v) { int e; (void)frexp(v, &e); return e; }
template <typename R>
__device__ __forceinline__ R re_div(C<R> D, C<R> u)
{
#pragma clang fp contract(off)
    const R m = fmax(fabs(u.x), fabs(u.y));
    if (m == R(0)) return R(0);
    const int e = -exponent_of(m);
    const R ux = scale2(u.x, e), uy = scale2(u.y, e), dx = scale2(D.x, e), dy = scale2(D.y, e);
    return (dx * ux + dy * uy) / (ux * ux + uy * uy);
}
template <typename R>
__device__ __forceinline__ R im_div(C<R> F, C<R> u)
{
#pragma clang fp contract(off)
    const R m = fmax(fabs(u.x), fabs(u.y));
    if (m == R(0)) return R(0);
    const int e = -exponent_of(m);
    const R ux = scale2(u.x, e), uy = scale2(u.y, e), fx = scale2(F.x, e), fy = scale2(F.y, e);
    return (fy * ux - fx * uy) / (ux * ux + uy * uy);
}

// MSD time derivative on a boundary node (Sec. 3.2, Eq. msdbc_ut): i w Psi_b with
// w = Im(F_{b-1} / Psi_{b-1}).  Contraction off, so that the products are rounded before any
// sum they enter, whichever kernel forms them.
template <typename R>
__device__ __forceinline__ C<R> msd_fb(R w, C<R> ub)
{
#pragma clang fp contract(off)
    return mk<R>(-w * ub.y, w * ub.x);
}

// K_tot accumulation of stages 2 and 3: K + 2F (2F is exact).
template <typename R>
__device__ __forceinline__ C<R> kacc(C<R> k, C<R> F)
{
#pragma clang fp contract(off)
    return mk<R>(fmar(R(2), F.x, k.x), fmar(R(2), F.y, k.y));
}

// base + ck * F (Sec. 3.1, the array updates of Eq. RK4).  When the master type
// is wider than the stage type the increment is rounded to the stage type first.
template <typename R, typename M>
__device__ __forceinline__ C<M> axpy_m(C<M> base, R ck, C<R> F)
{
#pragma clang fp contract(off)
    if constexpr (sizeof(M) == sizeof(R)) {
        return mk<M>(fmar(ck, F.x, base.x), fmar(ck, F.y, base.y));
    } else {
        const R ix = ck * F.x, iy = ck * F.y;
        return mk<M>(base.x + (M)ix, base.y + (M)iy);
    }
}

}  // namespace nlse
