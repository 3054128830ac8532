// Persistent 1D 2SHOC-RK4 solver: one workgroup keeps the whole field on chip
// and runs every RK4 step of the call in a single launch.
//
// Per stage (Sec. 2.1 Eqs. 2shoc1d-2shoc1d2, Sec. 3.1-3.2):
//   phase A  D_i = (Psi_{i+1} - 2 Psi_i + Psi_{i-1}) / h^2 on interior nodes (LDS);
//            boundary D_b: Dirichlet Eq. dbc_lap, or MSD Eq. msdbc_lap, which needs
//            D_{b-1}: the owner of the boundary node recomputes it from Psi.
//   phase B  Lap_i = (7/6) D_i - (1/12)(D_{i+1} + D_{i-1});  F_i = i[a Lap_i + (s|Psi_i|^2 - V_i) Psi_i];
//            boundary F_b: Dirichlet 0 (Eq. dbc_ut); MSD i Im(F_{b-1}/Psi_{b-1}) Psi_b (Eq. msdbc_ut),
//            with F_{b-1} recomputed by the boundary owner (interior first, boundary second).
//   phase C  the RK4 array operations of the stage; the next stage field is written to LDS.
// Psi^n (master precision), K_tot and V stay in registers of the owning thread for
// the whole launch; LDS holds the stage field and D.  HBM is touched only to load
// Psi^n at the start and store it at the end.
#include "onchip1d.h"

namespace nlse {

template <typename R> struct NPT1D;
template <> struct NPT1D<double> { static constexpr int v = 5; };   // 5 x 1024 nodes x 32 B = 160 KiB
template <> struct NPT1D<float> { static constexpr int v = 9; };    // 9 x 1024 nodes x 16 B = 144 KiB

constexpr int BS1D = 1024;

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
    const size_t lds = 2 * sizeof(C<R>) * (size_t)(a.L.nx + 1);
    // a launch that asks for more LDS than the device has fails with an error code
    (void)hipFuncSetAttribute((const void *)solve1d_kernel<R, M>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
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
