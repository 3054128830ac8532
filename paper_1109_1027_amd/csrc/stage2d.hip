// Fused RK4-stage kernel for the 2D NLSE with the per-axis 2SHOC Laplacian.
//
// One stage evaluates, on every interior node (Sec. 2.2 Eqs. 2d2shocMs1-2, Sec. 3.1):
//   step 1   D^x = delta_x^2 Psi,  D^y = delta_y^2 Psi
//   step 2   Lap = (7/6)(D^x + D^y) - (1/12)(D^x_{i+1} + D^x_{i-1} + D^y_{j+1} + D^y_{j-1})
//   RHS      F = i[a Lap + (s|Psi|^2 - V) Psi]
//   RK4      the stage's array operations of Eq. RK4 (see StageArgs)
// D never leaves the chip: D^y lives in registers (each lane owns one column and
// walks down its rows), D^x and the Psi row it is built from are exchanged
// through an LDS row buffer with a one-column halo.
//
// Boundary closure.  The per-axis form needs D^a on the face nodes normal to a.
// They are D^a_b = Lap_b - (tangential second difference), where Lap_b is the
// step-1 boundary value (Eq. dbc_lap, or Eq. msdbc_lap under MSD).  With these
// face values the per-axis and single-storage forms (Eq. 2d2shocs1-2) are
// algebraically identical.  Under Dirichlet the boundary values never change, so
// D^a_b are constants computed once per field (launch_boundary_d); under MSD
// msd.hip forms them from the stage's input, and updates the boundary nodes, in a
// launch before each stage launch.  Either way only boundary tiles read them.
//
// Tiling.  A wave owns 64 consecutive interior columns (aligned, one row segment
// = one coalesced access) and RW rows (RW = 4, 8 or 16: the tile variants the
// autotuner chooses from; every variant computes bit-identical results).  It loads RW + 4 rows of its columns
// (2-row halo for D^y at the tile's first/last rows), and one extra masked load
// brings the 2-column halo on each side for the RW rows.  Blocks of 4 waves
// take 4 consecutive tiles along x; blocks are remapped so that each XCD owns a
// contiguous band of tiles.
//
// Alternative Laplacians for comparison (StageArgs::stencil): the non-compact
// fourth-order stencil (-Psi_{+-2} + 16 Psi_{+-1} - 30 Psi) / (12 h^2) per axis,
// the one 2SHOC is measured against in Sec. 2.1 and Sec. 5, with the ghosts
// 2 Psi_b - Psi_{b+-1} + h^2 D^a_b one node beyond a face (their second difference at b
// is the face value of Eq. dbc_lap, so next to the boundary the stencil is the 2SHOC
// combination, as Sec. 2.1 shows it is inside); and the second-order
// central difference (CD) D^x + D^y.  Both read only what the 2SHOC tile already
// holds (two halo rows in registers, two halo columns in LDS).
#include "tile2d.h"

namespace nlse {

template <typename IN, typename R, typename M, int RW, int ST>
__global__ __launch_bounds__(256) void stage2d_kernel(StageArgs A, int64_t tiles_x, int64_t tiles_total)
{
    constexpr int NW = 4;
    __shared__ C<R> lds[NW][RW][TILE_W + 4];      // Psi rows, columns x0-2 .. x0+65
    __shared__ C<R> ldx[NW][RW][TILE_W + 2];      // D^x rows, columns x0-1 .. x0+64
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x) * NW + (threadIdx.x >> 6);
    stage2d_tile<IN, R, M, RW, NW, ST>(A, tile, tiles_x, tiles_total, lds, ldx);
}

template <typename IN, typename R, typename M, int RW, int ST>
static hipError_t launch_rw(const StageArgs &a, hipStream_t st)
{
    const int64_t tiles_x = (a.L.nx - 1 + 63) / 64;
    const int64_t tiles_y = (a.L.ny - 1 + RW - 1) / RW;
    const int64_t tiles = tiles_x * tiles_y;
    const int64_t blocks = (tiles + 3) / 4;
    hipLaunchKernelGGL((stage2d_kernel<IN, R, M, RW, ST>), dim3((unsigned)blocks), dim3(256), 0, st, a,
                       tiles_x, tiles);
    return hipGetLastError();
}

template <typename IN, typename R, typename M, int ST>
static hipError_t launch2s(const StageArgs &a, hipStream_t st)
{
    switch (a.variant) {
    case 0: return launch_rw<IN, R, M, 8, ST>(a, st);
    case 1: return launch_rw<IN, R, M, 4, ST>(a, st);
    case 2: return launch_rw<IN, R, M, 16, ST>(a, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename IN, typename R, typename M>
static hipError_t launch2v(const StageArgs &a, hipStream_t st)
{
    switch (a.stencil) {
    case 0: return launch2s<IN, R, M, 0>(a, st);
    case 1: return launch2s<IN, R, M, 1>(a, st);
    case 2: return launch2s<IN, R, M, 2>(a, st);
    default: return hipErrorInvalidValue;
    }
}

int stage2d_variants() { return 3; }

hipError_t launch_stage2d(Prec prec, const StageArgs &a, hipStream_t st)
{
    switch (prec) {
    case P_F64: return launch2v<double, double, double>(a, st);
    case P_F32: return launch2v<float, float, float>(a, st);
    default:
        if (a.stage == 1) return launch2v<double, float, double>(a, st);
        return launch2v<float, float, double>(a, st);
    }
}

}  // namespace nlse
