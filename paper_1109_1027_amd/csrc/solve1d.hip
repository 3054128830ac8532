// Persistent 1D 2SHOC-RK4 solver: one workgroup keeps the whole field on chip
// (in registers, see onchip1d.h for the scheme) and runs every RK4 step of the
// call in a single launch.
#include "onchip1d.h"

namespace nlse {

template <typename R> struct NPT1D;
template <> struct NPT1D<double> { static constexpr int v = 10; };   // 512 threads x 10 nodes
template <> struct NPT1D<float> { static constexpr int v = 18; };    // 512 threads x 18 nodes

constexpr int BS1D = 512;

template <typename R, typename M>
__global__ __launch_bounds__(BS1D) void solve1d_kernel(Solve1DArgs A)
{
    extern __shared__ unsigned char smem_raw[];
    solve1d_onchip<R, M, BS1D, NPT1D<R>::v>(A, smem_raw);
}

int64_t solve1d_max_nodes(Prec prec)
{
    return (int64_t)BS1D * (prec == P_F64 ? NPT1D<double>::v : NPT1D<float>::v);
}

template <typename R, typename M>
static hipError_t launch1d(const Solve1DArgs &a, hipStream_t st)
{
    const size_t lds = onchip1d_lds<R, BS1D>();
    hipLaunchKernelGGL((solve1d_kernel<R, M>), dim3(1), dim3(BS1D), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_solve1d(Prec prec, const Solve1DArgs &a, hipStream_t st)
{
    if (a.L.nx + 1 > solve1d_max_nodes(prec)) return hipErrorInvalidValue;
    switch (prec) {
    case P_F64: return launch1d<double, double>(a, st);
    case P_F32: return launch1d<float, float>(a, st);
    default: return launch1d<float, double>(a, st);
    }
}

}  // namespace nlse
