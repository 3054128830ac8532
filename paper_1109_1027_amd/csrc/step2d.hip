// Whole-step RK4 kernel for the 2D NLSE with the per-axis 2SHOC Laplacian.
//
// One launch advances Psi^n to Psi^{n+1}: the four stages of Eq. RK4 (Sec. 3.1),
// each the per-axis 2SHOC Laplacian of Sec. 2.2 (Eqs. 2d2shocMs1-2) fused with
// the right-hand side.  The point-wise arithmetic is the stage kernel's
// (point.h), so the result is bit-identical to four stage launches, but only
// Psi^n and V are read and only Psi^{n+1} is written: the stage fields, D^x,
// D^y and K_tot never leave the registers of the wave that produces them.
//
// Scheme.  A wave owns a strip of 64 consecutive columns and walks down a
// segment of rows.  Stage s needs stage s-1 within two rows and two columns,
// so the four stages run as a pipeline skewed by two rows: when row j of Psi^n
// arrives, stage 1 produces row j-2 of its output, stage 2 row j-4, stage 3
// row j-6 and stage 4 row j-8 of Psi^{n+1}.  Along y each stage keeps its last
// three input rows and three D^y rows in registers; along x the neighbours come
// from the adjacent lanes through DPP wave shifts (no LDS exchange, no barriers).  The
// valid columns shrink by two per side and stage, so the middle 48 of the 64
// lanes produce Psi^{n+1}: neighbouring strips overlap by 16 columns and
// neighbouring segments by 16 rows of recomputed halo.
//
// Register rings.  Psi^n, V and K_tot are needed 2, 4, 6 and 8 rows after they
// arrive, so they sit in 9-row rings; the per-stage row queues have length 3.
// The row loop is unrolled by 9, which makes every ring index a constant.
//
// Boundary closure as in the stage kernel: boundary nodes keep their Dirichlet
// values in every stage, and the face-normal D^a_b come from the precomputed
// face arrays.  Lanes and rows outside the grid feed no interior node.
#include "wave2d.h"

namespace nlse {

namespace {

constexpr int NW = 4;      // waves per block (independent)

template <typename R, typename M, int Q, int PD, int ST>
__global__ __launch_bounds__(256) void step2d_kernel(Step2DArgs A, int strips, int waves)
{
    // Wave-private staging (written and read by the same wave only, so no barrier is needed).
    __shared__ wave2d::Staging<R, Q> stg[NW];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int w = (int)xcd_remap(blockIdx.x, gridDim.x) * NW + wv;
    if (w >= waves) return;                 // whole waves only; the kernel has no barriers
    wave2d::step2d_wave<R, M, Q, PD, ST>(A, w % strips, w / strips, threadIdx.x & 63, stg[wv]);
}

template <typename R, typename M, int ST, int Q, int PD = 1>
hipError_t launch_q(const Step2DArgs &a, hipStream_t st)
{
    if (a.L.total >= (int64_t(1) << 31)) return hipErrorInvalidValue;   // 32-bit offsets
    const int strips = wave2d::strips(a.L.nx);
    const int segs = wave2d::segments<Q>(a.L.ny);
    const int waves = strips * segs;
    const int blocks = (waves + NW - 1) / NW;
    hipLaunchKernelGGL((step2d_kernel<R, M, Q, PD, ST>), dim3(blocks), dim3(64 * NW), 0, st, a, strips, waves);
    return hipGetLastError();
}

template <typename R, typename M, int ST>
hipError_t launch_v(const Step2DArgs &a, hipStream_t st)
{
    switch (a.variant) {
    case 0: return launch_q<R, M, ST, 5>(a, st);    // 29-row segments
    case 1: return launch_q<R, M, ST, 4>(a, st);    // 20
    case 2: return launch_q<R, M, ST, 6>(a, st);    // 38
    case 3: return launch_q<R, M, ST, 8>(a, st);    // 56
    case 4: return launch_q<R, M, ST, 3>(a, st);    // 11 (small grids: more, shorter waves)
    case 5: return launch_q<R, M, ST, 7>(a, st);    // 47
    case 6: return launch_q<R, M, ST, 5, 2>(a, st);  // 29, two rows of Psi^n in flight (pays off in mixed)
    default: return hipErrorInvalidValue;
    }
}

template <typename R, typename M>
hipError_t launch_s(const Step2DArgs &a, hipStream_t st)
{
    switch (a.stencil) {
    case 0: return launch_v<R, M, 0>(a, st);
    case 1: return launch_v<R, M, 1>(a, st);
    case 2: return launch_v<R, M, 2>(a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int step2d_variants() { return 7; }

hipError_t launch_step2d(Prec prec, const Step2DArgs &a, hipStream_t st)
{
    switch (prec) {
    case P_F64: return launch_s<double, double>(a, st);
    case P_F32: return launch_s<float, float>(a, st);
    default: return launch_s<float, double>(a, st);
    }
}

}  // namespace nlse
