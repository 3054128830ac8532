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
// three input rows and three D^y rows in registers; along x each stage input row
// also goes through a wave-private LDS ring, read two rows after it was written,
// and the neighbours of D^x come from the adjacent lanes through DPP wave shifts
// (no barriers).  The valid columns shrink by two per side and stage, so the
// middle 48 of the 64 lanes produce Psi^{n+1}: neighbouring strips overlap by 16
// columns and neighbouring segments by 16 rows of recomputed halo.
//
// Register rings.  Psi^n, V and K_tot are needed 2, 4, 6 and 8 rows after they
// arrive, so they sit in 9-row rings; the per-stage row queues have length 3.
// The row loop is unrolled by 9, which makes every ring index a constant.
//
// Boundary closure as in the stage kernel: boundary nodes keep their Dirichlet
// values in every stage, and the face-normal D^a_b come from the precomputed
// face arrays.  Lanes and rows outside the grid feed no interior node.
//
// This header holds the kernels and their launch templates; each precision and boundary rule
// instantiates them in a translation unit of its own (step2d_<prec>.hip, step2d_msd_<prec>.hip),
// so the build compiles them in parallel, and step2d.hip dispatches.
#pragma once

#include "wave2d.h"

namespace nlse {

namespace {


constexpr int NW = 4;      // waves per block (independent)

// MSD: the edge strips' segments have ng_e <= Q row groups (see launch_q).
template <typename R, typename M, int Q, int PD, int ST, bool MSD>
__device__ __forceinline__ void step2d_body(const Step2DArgs &A, int strips, int waves, int segs, int segs_e,
                                            int ng_e)
{
    // Wave-private staging (written and read by the same wave only, so no barrier is needed).
    __shared__ wave2d::Staging<R, Q> stg[NW];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int strip, seg;
    if constexpr (MSD) {
        // The edge strips carry the face closures and run longest: their tasks go to the blocks
        // dispatched first, whose waves are the older of the two on their SIMD and issue first.
        // The edge strips also get shorter segments (ng_e row groups), so that they end with the rest.
        const int w = (int)blockIdx.x * NW + wv;
        if (w >= waves) return;
        const int ne = strips > 1 ? 2 : 1;
        if (w < ne * segs_e) {
            strip = (w % ne) ? strips - 1 : 0;
            seg = w / ne;
            wave2d::step2d_wave<R, M, Q, PD, ST, MSD>(A, strip, seg, threadIdx.x & 63, stg[wv], ng_e);
            return;
        }
        const int k = w - ne * segs_e;
        strip = 1 + k % (strips - 2);
        seg = k / (strips - 2);
        const int xs = 1 + wave2d::SW * strip - wave2d::HALO;
        if (xs > 0 && xs + 63 < (int)A.L.nx) {   // no face column among the wave's lanes
            if (wave2d::meets_face_rows((int)A.L.ny, seg, Q))
                wave2d::step2d_wave<R, M, Q, PD, ST, MSD, false>(A, strip, seg, threadIdx.x & 63, stg[wv]);
            else   // nor a face row: the closure code of rows 0 and ny compiled out too
                wave2d::step2d_wave<R, M, Q, PD, ST, MSD, false, false>(A, strip, seg, threadIdx.x & 63, stg[wv]);
            return;
        }
    } else {
        const int w = (int)xcd_remap(blockIdx.x, gridDim.x) * NW + wv;
        if (w >= waves) return;             // whole waves only; the kernel has no barriers
        strip = w % strips;
        seg = w / strips;
        (void)segs;
        (void)segs_e;
        (void)ng_e;
    }
    wave2d::step2d_wave<R, M, Q, PD, ST, MSD>(A, strip, seg, threadIdx.x & 63, stg[wv]);
}

template <typename R, typename M, int Q, int PD, int ST, bool MSD>
__global__ __launch_bounds__(256) void step2d_kernel(Step2DArgs A, int strips, int waves)
{
    step2d_body<R, M, Q, PD, ST, MSD>(A, strips, waves, 0, 0, Q);
}

// The MSD instances hold a few more values; the bound keeps two waves per SIMD (the FP64 one
// spills a few scalars of its boundary rows).
template <typename R, typename M, int Q, int PD, int ST, bool MSD>
__global__ __launch_bounds__(256, 2) void step2d_msd_kernel(Step2DArgs A, int strips, int waves, int segs, int segs_e,
                                                            int ng_e)
{
    step2d_body<R, M, Q, PD, ST, MSD>(A, strips, waves, segs, segs_e, ng_e);
}

template <typename R, typename M, int ST, bool MSD, int Q, int PD = 1>
hipError_t launch_q(const Step2DArgs &a, hipStream_t st)
{
    if (a.L.total >= (int64_t(1) << 31)) return hipErrorInvalidValue;   // 32-bit offsets
    const int strips = wave2d::strips(a.L.nx);
    const int segs = wave2d::segments<Q>(a.L.ny + (MSD ? 1 : 0));   // MSD: rows 1 .. ny
    if constexpr (MSD) {
        // edge strips: about half as many row groups (their waves carry the face closures)
        const int ng_e = Q > 4 ? (Q + 1) / 2 : Q;
        const int segs_e = wave2d::segments_ng(a.L.ny + 1, ng_e);
        const int ne = strips > 1 ? 2 : 1;
        const int waves = ne * segs_e + (strips - ne) * segs;
        const int blocks = (waves + NW - 1) / NW;
        hipLaunchKernelGGL((step2d_msd_kernel<R, M, Q, PD, ST, MSD>), dim3(blocks), dim3(64 * NW), 0, st, a, strips,
                           waves, segs, segs_e, ng_e);
    } else {
        const int waves = strips * segs;
        const int blocks = (waves + NW - 1) / NW;
        hipLaunchKernelGGL((step2d_kernel<R, M, Q, PD, ST, MSD>), dim3(blocks), dim3(64 * NW), 0, st, a, strips, waves);
    }
    return hipGetLastError();
}

template <typename R, typename M, int ST, bool MSD = false>
hipError_t launch_v(const Step2DArgs &a, hipStream_t st)
{
    switch (a.variant) {
    case 0: return launch_q<R, M, ST, MSD, 5>(a, st);    // 29-row segments
    case 1: return launch_q<R, M, ST, MSD, 4>(a, st);    // 20
    case 2: return launch_q<R, M, ST, MSD, 6>(a, st);    // 38
    case 3: return launch_q<R, M, ST, MSD, 8>(a, st);    // 56
    case 4: return launch_q<R, M, ST, MSD, 3>(a, st);    // 11 (small grids: more, shorter waves)
    case 5: return launch_q<R, M, ST, MSD, 7>(a, st);    // 47
    case 6: return launch_q<R, M, ST, MSD, 5, 2>(a, st);  // 29, two rows of Psi^n in flight (pays off in mixed)
    default: return hipErrorInvalidValue;
    }
}

template <typename R, typename M>
hipError_t launch_dirichlet(const Step2DArgs &a, hipStream_t st)
{
    switch (a.stencil) {
    case 0: return launch_v<R, M, 0>(a, st);
    case 1: return launch_v<R, M, 1>(a, st);
    case 2: return launch_v<R, M, 2>(a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

}  // namespace nlse
