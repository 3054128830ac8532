// Host-side launchers of the device kernels (one translation unit per family).
#pragma once

#include "common.h"

namespace nlse {

enum Prec { P_F64 = 0, P_F32 = 1, P_MIXED = 2 };

// Arguments of one fused RK4-stage launch (2D and 3D share the struct).
//   stage 1: in = Psi^n            K = F          out = Psi^n + (k/2) F
//   stage 2: in = Psi_tmp          K += 2F        out = Psi^n + (k/2) F
//   stage 3: in = Psi_tmp          K += 2F        out = Psi^n + k F
//   stage 4: in = Psi_tmp          Psi^n = Psi^n + (k/6)(K + F)
// Only interior nodes are written; boundary nodes of every stage field hold the
// fixed Dirichlet values (under MSD, launch_msd_stage writes them).
struct StageArgs {
    const void *in;     // stencil input field
    void *out;          // stage output (stages 1-3)
    void *psin;         // master Psi^n
    void *K;            // K_tot
    const void *V;      // potential (real) or nullptr
    const void *DB[3];  // boundary-face normal second differences, per axis [2][face nodes]
    Layout L;
    Coeffs c;
    int stage;
    int variant;        // tile-shape variant (see stage2d_variants / stage3d_variants)
    int stencil;        // 0 2SHOC, 1 non-compact fourth order, 2 second-order CD
};

// 2D fused stage kernel: per-axis 2SHOC, one 64-column x RW-row tile per wave.
hipError_t launch_stage2d(Prec prec, const StageArgs &a, hipStream_t st);
int stage2d_variants();
// 3D fused stage kernel (2.5D: x-y tile in LDS, march along z).
hipError_t launch_stage3d(Prec prec, const StageArgs &a, hipStream_t st);
int stage3d_variants();

// 2D whole-step kernel: all four RK4 stages of one step in one launch (see
// step2d.hip).  Reads the master Psi^n from psi_in and writes the interior of
// Psi^{n+1} to psi_out, a different buffer whose boundary nodes already hold
// the (fixed) Dirichlet values.  K_tot and the stage fields stay on chip.
struct Step2DArgs {
    const void *psi_in;
    void *psi_out;
    const void *V;       // potential (real, stage type); never nullptr (zeros when V = 0)
    const void *DB[2];   // boundary-face normal second differences (as in StageArgs)
    Layout L;
    Coeffs c;            // ck unused
    double ck[4];        // k/2, k/2, k, k/6
    int variant;
    int stencil;         // 0 2SHOC, 1 non-compact fourth order, 2 second-order CD
    int msd;             // 1: MSD boundary (2SHOC only; boundary nodes of psi_out written too, DB unused)
};
hipError_t launch_step2d(Prec prec, const Step2DArgs &a, hipStream_t st);
// its parts, one translation unit each (step2d_<prec>.hip: Dirichlet, every Laplacian;
// step2d_msd_<prec>.hip: MSD)
hipError_t launch_step2d_f64(const Step2DArgs &a, hipStream_t st);
hipError_t launch_step2d_f32(const Step2DArgs &a, hipStream_t st);
hipError_t launch_step2d_mixed(const Step2DArgs &a, hipStream_t st);
hipError_t launch_step2d_msd_f64(const Step2DArgs &a, hipStream_t st);
hipError_t launch_step2d_msd_f32(const Step2DArgs &a, hipStream_t st);
hipError_t launch_step2d_msd_mixed(const Step2DArgs &a, hipStream_t st);
int step2d_variants();

// 3D step as two launches of two fused stages each (see step3d.hip): pair 1 reads
// psin (Psi^n) and V and writes K and B (the stage-2 field); pair 2 reads B, K,
// psin and V and writes Psi^{n+1} to psi_out, a different buffer whose boundary
// nodes already hold the (fixed) Dirichlet values.
struct Step3DArgs {
    const void *psin;
    void *psi_out;
    void *K;
    void *B;
    const void *V;       // potential (real, stage type) or nullptr
    const void *DB[3];   // boundary-face normal second differences (as in StageArgs)
    Layout L;
    Coeffs c;            // ck unused
    double ck[4];        // k/2, k/2, k, k/6
    int variant;
};
hipError_t launch_step3d(Prec prec, const Step3DArgs &a, hipStream_t st);
int step3d_variants();

// 1D persistent solver: one workgroup holds the whole field on chip and runs
// nsteps RK4 steps in one launch.
struct Solve1DArgs {
    void *psin;          // master Psi^n (in/out)
    const void *V;       // real potential or nullptr
    Layout L;
    Coeffs c;            // ck unused; k, k/2, k/6 below
    double k, k2, k6;
    int64_t nsteps;
    int msd;             // 1: MSD boundary, 0: Dirichlet
    int variant;         // 0: 512 threads, 1: 256 threads, 2 / 3: 512 threads with at most 4 / 3 nodes each
    int stencil;         // 0 2SHOC, 1 non-compact fourth order, 2 second-order CD (Dirichlet only)
};
hipError_t launch_solve1d(Prec prec, const Solve1DArgs &a, hipStream_t st);
int64_t solve1d_max_nodes(Prec prec);               // the largest field of variant 0
int solve1d_variants(Prec prec, int64_t nodes);     // variants 0 .. that hold `nodes`

// Boundary-face normal second differences D^a_b = Lap_b - sum_{tangential} delta^2 Psi_b
// for the per-axis 2SHOC (Dirichlet, 2D/3D), from the master field.
hipError_t launch_boundary_d(Prec prec, const void *psin, const void *V, const Layout &L,
                             const Coeffs &c, void *DB[3], hipStream_t st);

// MSD boundary in 2D/3D (msd.hip).  Face values D^a_b of the per-axis form from the MSD
// step-1 closure of the field `in` (master = true: `in` is the master field, else a
// stage field) into DB; the boundary part of one RK4 stage, launched before the
// interior launch with the same StageArgs: the face values of a.in into DB, and F_b
// with the stage's RK4 array operations on every boundary node; and the bound's
// boundary term max (h^2/a)|F_{b-1}/Psi_{b-1}| of the master field into dev_out (face
// values first).
hipError_t launch_msd_faces(Prec prec, bool master, const void *in, const void *V, const Layout &L,
                            const Coeffs &c, void *const DB[3], hipStream_t st);
hipError_t launch_msd_stage(Prec prec, const StageArgs &a, void *const DB[3], hipStream_t st);
hipError_t launch_msd_bound(Prec prec, const void *psin, const void *V, const void *const DB[3], const Layout &L,
                            const Coeffs &c, double h2a, double *dev_out, hipStream_t st);

// 1D boundary closure on the device (aux.hip): D_b of both ends (Eq. dbc_lap, or Eq. msdbc_lap
// when msd) into DB ([2] stage complex), and under MSD the bound's boundary term
// max (h^2/a)|F_{b-1}/Psi_{b-1}| into *bound_out (may be nullptr).
hipError_t launch_edges1d(Prec prec, const void *psin, const void *V, const Layout &L, const Coeffs &c, bool msd,
                          double h2a, void *DB, double *bound_out, hipStream_t st);

// Copy the master field into a stage field, converting to the stage type.
hipError_t launch_master_to_stage(Prec prec, const void *psin, void *dst, const Layout &L,
                                  hipStream_t st);

// Deterministic FP64 reductions.  `partials` must hold reduce_partials() doubles
// (times 2 for minmax); the result is written to dev_out (device) and is
// bitwise reproducible for a given layout.
int reduce_partials();
// dev_out[0] = scale * (sum of |Psi|^2 over every node).
hipError_t launch_mass(Prec prec, const void *psin, const Layout &L, double *partials,
                       double *dev_out, hipStream_t st, double scale = 1.0);
hipError_t launch_energy(Prec prec, const void *psin, const void *V, const void *const DB[3],
                         const Layout &L, const Coeffs &c, double *partials, double *dev_out,
                         hipStream_t st);
// dev_out[0] = min over interior of (s|Psi|^2 - V), dev_out[1] = max.
hipError_t launch_minmax_nonlin(Prec prec, const void *psin, const void *V, const Layout &L,
                                double s, double *partials, double *dev_out, hipStream_t st);

}  // namespace nlse
