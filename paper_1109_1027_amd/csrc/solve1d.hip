// Persistent 1D 2SHOC-RK4 solver: one workgroup keeps the whole field on chip
// (in registers, see onchip1d.h for the scheme) and runs every RK4 step of the
// call in a single launch.  Variants, in decreasing capacity: 512 threads with up
// to NPT1D nodes each, 256 threads with as many, and 512 threads with at most 4 or
// 3 (fields of up to 2048 / 1536 nodes).  Every slot of the register arrays costs
// instructions whether a thread uses it or not, so the tightest bound is fastest.
#include "onchip1d.h"

namespace nlse {

template <typename R> struct NPT1D;
template <> struct NPT1D<double> { static constexpr int v = 10; };   // nodes per thread at most
template <> struct NPT1D<float> { static constexpr int v = 18; };

template <typename R, typename M, int BS, int NPT, int ST>
__global__ __launch_bounds__(BS) void solve1d_kernel(Solve1DArgs A)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    solve1d_onchip<R, M, BS, NPT, ST>(A, smem_raw);
}

static int npt_of(Prec prec) { return prec == P_F64 ? NPT1D<double>::v : NPT1D<float>::v; }

// Largest field of each variant.
static int64_t capacity(Prec prec, int variant)
{
    switch (variant) {
    case 0: return 512 * (int64_t)npt_of(prec);
    case 1: return 256 * (int64_t)npt_of(prec);
    case 2: return 512 * 4;
    case 3: return 512 * 3;
    default: return 0;
    }
}

int64_t solve1d_max_nodes(Prec prec) { return capacity(prec, 0); }

int solve1d_variants(Prec prec, int64_t nodes)
{
    int n = 0;
    while (n < 4 && capacity(prec, n) >= nodes) ++n;
    return n;
}

template <typename R, typename M, int BS, int NPT>
static hipError_t launch1d(const Solve1DArgs &a, hipStream_t st)
{
    const size_t lds = onchip1d_lds<R, BS>();
    switch (a.stencil) {
    case 0: hipLaunchKernelGGL((solve1d_kernel<R, M, BS, NPT, 0>), dim3(1), dim3(BS), lds, st, a); break;
    case 1: hipLaunchKernelGGL((solve1d_kernel<R, M, BS, NPT, 1>), dim3(1), dim3(BS), lds, st, a); break;
    case 2: hipLaunchKernelGGL((solve1d_kernel<R, M, BS, NPT, 2>), dim3(1), dim3(BS), lds, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename R, typename M>
static hipError_t launch1d_v(const Solve1DArgs &a, hipStream_t st)
{
    switch (a.variant) {
    case 0: return launch1d<R, M, 512, NPT1D<R>::v>(a, st);
    case 1: return launch1d<R, M, 256, NPT1D<R>::v>(a, st);
    case 2: return launch1d<R, M, 512, 4>(a, st);
    case 3: return launch1d<R, M, 512, 3>(a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve1d(Prec prec, const Solve1DArgs &a, hipStream_t st)
{
    if (a.variant < 0 || a.variant >= solve1d_variants(prec, a.L.nx + 1)) return hipErrorInvalidValue;
    if (a.stencil != 0 && a.msd) return hipErrorInvalidValue;   // the MSD closure is the 2SHOC one
    switch (prec) {
    case P_F64: return launch1d_v<double, double>(a, st);
    case P_F32: return launch1d_v<float, float>(a, st);
    default: return launch1d_v<float, double>(a, st);
    }
}

}  // namespace nlse
