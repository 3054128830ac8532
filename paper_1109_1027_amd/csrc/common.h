// Shared device/host definitions of the gfx950 2SHOC-RK4 library.
//
// Device layout of every field (padded, x fastest):
//   element (x, y, z) of a field with nx, ny, nz intervals lives at
//     ((z * py) + y) * px + x + ox
//   ox = 63 puts the first interior column (x = 1) on a 64-element boundary and
//   px is a multiple of 64, so each wave's 64-lane row segment of interior
//   nodes is one aligned, fully coalesced access (1 KiB for complex128,
//   512 B for complex64).  Unused axes have one node.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace nlse {

template <typename R> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename R> using C = typename cplx_t<R>::type;

// Loads and stores of device memory through the global address space.  A pointer that a
// kernel reads from memory (the batched launch takes its instances' fields from a table) is
// generic to the compiler, and generic (flat) accesses are counted together with LDS accesses:
// each wait for an LDS read would then also wait for every row load in flight.  These keep
// such accesses global whatever the compiler knows of the pointer.
typedef float dev_f2 __attribute__((ext_vector_type(2)));
typedef double dev_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float dev_ld(const float *p) { return *(const __attribute__((address_space(1))) float *)p; }
__device__ __forceinline__ double dev_ld(const double *p) { return *(const __attribute__((address_space(1))) double *)p; }
__device__ __forceinline__ float2 dev_ld(const float2 *p)
{
    const dev_f2 v = *(const __attribute__((address_space(1))) dev_f2 *)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 dev_ld(const double2 *p)
{
    const dev_d2 v = *(const __attribute__((address_space(1))) dev_d2 *)p;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void dev_st(float2 *p, float2 v)
{
    const dev_f2 w = {v.x, v.y};
    *(__attribute__((address_space(1))) dev_f2 *)p = w;
}
__device__ __forceinline__ void dev_st(double2 *p, double2 v)
{
    const dev_d2 w = {v.x, v.y};
    *(__attribute__((address_space(1))) dev_d2 *)p = w;
}

template <typename R>
__host__ __device__ __forceinline__ C<R> mk(R x, R y) { C<R> r; r.x = x; r.y = y; return r; }

template <typename To, typename From>
__host__ __device__ __forceinline__ C<To> cvt(const C<From> &v) { return mk<To>((To)v.x, (To)v.y); }

template <typename R>
__device__ __forceinline__ C<R> cadd(C<R> u, C<R> v) { return mk<R>(u.x + v.x, u.y + v.y); }
template <typename R>
__device__ __forceinline__ C<R> csub(C<R> u, C<R> v) { return mk<R>(u.x - v.x, u.y - v.y); }
template <typename R>
__device__ __forceinline__ C<R> cscale(R k, C<R> u) { return mk<R>(k * u.x, k * u.y); }
template <typename R>
__device__ __forceinline__ C<R> czero() { return mk<R>(R(0), R(0)); }

// settle(v): an empty asm statement that reads v, so v (and the load it came from) must be
// complete at this point.  The vector-memory wait counter covers loads and stores in issue
// order; a marching kernel settles its prefetched values before it issues the plane's
// stores, so that a later wait for the prefetch never waits for those stores as well.
__device__ __forceinline__ void settle(float v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void settle(double v) { asm volatile("" ::"v"(v)); }
__device__ __forceinline__ void settle(const float2 &v) { asm volatile("" ::"v"(v.x), "v"(v.y)); }
__device__ __forceinline__ void settle(const double2 &v) { asm volatile("" ::"v"(v.x), "v"(v.y)); }

struct Layout {
    int dim;
    int64_t nx, ny, nz;   // intervals per axis (0 for unused axes)
    int64_t px;           // elements per row (multiple of 64)
    int64_t py;           // rows per plane
    int64_t ox;           // position of node x = 0 inside its row
    int64_t total;        // elements per field

    __host__ __device__ __forceinline__ int64_t idx(int64_t x, int64_t y, int64_t z) const {
        return (z * py + y) * px + x + ox;
    }
    __host__ __device__ __forceinline__ int64_t interior() const {
        int64_t r = nx - 1;
        if (dim > 1) r *= (ny - 1);
        if (dim > 2) r *= (nz - 1);
        return r;
    }
};

inline Layout make_layout(int dim, const int64_t n[3]) {
    Layout L;
    L.dim = dim;
    L.nx = n[0];
    L.ny = dim > 1 ? n[1] : 0;
    L.nz = dim > 2 ? n[2] : 0;
    L.ox = 63;
    L.px = ((L.ox + L.nx + 1 + 63) / 64) * 64;
    L.py = L.ny + 1;
    L.total = L.px * L.py * (L.nz + 1);
    return L;
}

// Stencil and RK4 coefficients for one stage, in double; kernels convert them
// to their arithmetic type.  ih2 = 1/h^2, c76 = 7/6, c112 = 1/12 (Eq. 2shoc1d2).
struct Coeffs {
    double a, s, ih2, c76, c112, ia;   // ia = 1/a (boundary rule)
    double ck;                          // k/2, k/2, k, k/6 for stages 1..4
};

// Blocks are handed to the 8 XCDs round-robin (block b -> XCD b % 8).  Map the
// hardware block index to a logical tile index so that each XCD works on one
// contiguous range of tiles: neighbouring tiles, which read each other's halo
// rows, then share that XCD's L2.  A bijection on [0, nb).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t q = nb / 8, r = nb % 8;
    const int64_t k = b % 8, i = b / 8;
    return k < r ? k * (q + 1) + i : r * (q + 1) + (k - r) * q + i;
}

}  // namespace nlse
