// Neighbour exchange inside a wave through DPP (data-parallel primitives) lane
// shifts, shared by the register-resident 1D and 2D kernels.
#pragma once

#include "common.h"

namespace nlse {

// DPP wave shifts: wave_shr:1 delivers lane i-1's value to lane i, wave_shl:1
// lane i+1's; lanes shifted in from outside the wave read zero (bound_ctrl).
__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float lane_prev(float v) { return __int_as_float(dpp_prev(__float_as_int(v))); }
__device__ __forceinline__ float lane_next(float v) { return __int_as_float(dpp_next(__float_as_int(v))); }
__device__ __forceinline__ double lane_prev(double v)
{
    return __hiloint2double(dpp_prev(__double2hiint(v)), dpp_prev(__double2loint(v)));
}
__device__ __forceinline__ double lane_next(double v)
{
    return __hiloint2double(dpp_next(__double2hiint(v)), dpp_next(__double2loint(v)));
}
template <typename R>
__device__ __forceinline__ C<R> clane_prev(C<R> v) { return mk<R>(lane_prev(v.x), lane_prev(v.y)); }
template <typename R>
__device__ __forceinline__ C<R> clane_next(C<R> v) { return mk<R>(lane_next(v.x), lane_next(v.y)); }

}  // namespace nlse
