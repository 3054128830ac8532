"""GPU parity of the modulus-squared Dirichlet (MSD) boundary in 2D and 3D against the oracle.

Under MSD (Sec. 3.2, Eqs. msdbc_lap, msdbc_ut; b-1 the closest interior node, the diagonal one on
edges and corners) every RK4 stage runs the face-value launch, the interior stage kernel and the
boundary update.  Tolerances as for Dirichlet: relative L2 over all nodes <= 1e-12 (FP64) and
<= 1e-4 (FP32, mixed) after the whole run.  Sizes span several 64-column tiles with ragged tails.
"""
import sys

import numpy as np
import pytest

import nlse_inputs as I
from parity_util import line_err, rel

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-4, "mixed": 1e-4}


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1109_1027_amd as P
    P.load()
    return P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def vortex_case(n=150):
    g = I.grid(2, n, -20.0, 20.0)
    return g, I.background_vortices(g, pairs=2, seed=11)


def ring_case(n=40):
    g = I.grid(3, n, -8.0, 8.0)
    return g, I.background_ring(g, ring_radius=3.0)


def gpu_run(gpu, dim, n, h, psi, prec, nsteps, dt, variant=None, a=0.5, s=-1.0):
    sol = gpu.Solver(dim, n, h, a, s, None, "msd", prec)
    sol.set_field(psi.astype(sol.dtype))
    if variant is not None:
        sol.variant = variant
    sol.step(nsteps, dt)
    return sol.get_field(), sol


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
def test_msd_2d_vortex_pairs(gpu, orc, prec):
    g, psi = vortex_case()
    P = orc.Problem(2, g.n, g.h, 0.5, -1.0, bc="msd")
    dt = 0.5 * P.max_dt(psi)
    say(f"[case] msd 2d vortices n={g.n} prec={prec} steps=40 dt={dt:.6g}")
    out, sol = gpu_run(gpu, 2, g.n, g.h, psi, prec, 40, dt)
    ref = P.rk4(psi, 40, dt)
    e = rel(out, ref)
    say(f"  rel L2 = {e:.3e}")
    assert e <= TOL[prec]
    assert line_err(out, ref) <= TOL[prec]
    # the boundary moved (the rule is live) yet kept its density
    b = g.boundary_mask()
    assert np.max(np.abs(ref[b] - psi[b])) > 1e-3
    assert np.max(np.abs(np.abs(np.asarray(out, np.complex128)[b]) ** 2 - np.abs(psi[b]) ** 2)) < 1e-4
    sol.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
def test_msd_3d_ring(gpu, orc, prec):
    g, psi = ring_case()
    P = orc.Problem(3, g.n, g.h, 0.5, -1.0, bc="msd")
    dt = 0.5 * P.max_dt(psi)
    say(f"[case] msd 3d ring n={g.n} prec={prec} steps=10 dt={dt:.6g}")
    out, sol = gpu_run(gpu, 3, g.n, g.h, psi, prec, 10, dt)
    ref = P.rk4(psi, 10, dt)
    e = rel(out, ref)
    say(f"  rel L2 = {e:.3e}")
    assert e <= TOL[prec]
    assert line_err(out, ref) <= TOL[prec]
    sol.close()


def test_msd_2d_non_square_dark_plane(gpu, orc):
    """Non-square grid (nx = 64, ny = 16), steep density at the x = lo face."""
    n, psi = I.dark_plane(2, 0.25, width=4.0)
    P = orc.Problem(2, n, 0.25, 0.5, -1.0, bc="msd")
    nst, dt = orc.steps_for(1.0, P.max_dt(psi))
    say(f"[case] msd 2d dark plane n={n} steps={nst}")
    out, sol = gpu_run(gpu, 2, n, 0.25, psi, "f64", nst, dt)
    ref = P.rk4(psi, nst, dt)
    assert rel(out, ref) <= 1e-12
    assert line_err(out, ref) <= 1e-12
    _, exact = I.dark_plane(2, 0.25, t=1.0, width=4.0)
    assert rel(out, exact) < 1e-4   # the oracle's fourth-order error level at this h
    sol.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("width", [7.875, 0.5])
def test_msd_2d_faces_filling_whole_blocks(gpu, orc, prec, width):
    """The 2D boundary launch runs one-wave blocks: faces of exactly 64 and 128 nodes (no partial
    block), and a 5-node face (less than one block), on a perturbed dark plane."""
    h = 0.125
    n, psi = I.dark_plane(2, h, lo=-8.0, hi=7.875, width=width)   # 127 x 63 or 127 x 4 intervals
    rng = np.random.default_rng(5)
    psi = psi + 1e-3 * (rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))
    P = orc.Problem(2, n, h, 0.5, -1.0, bc="msd")
    dt = 0.5 * P.max_dt(psi)
    say(f"[case] msd 2d whole-block faces n={n} {prec}")
    out, sol = gpu_run(gpu, 2, n, h, psi, prec, 20, dt)
    sol.close()
    ref = P.rk4(psi, 20, dt)
    assert rel(out, ref) <= TOL[prec]
    assert line_err(out, ref) <= TOL[prec]


def test_msd_3d_non_cubic(gpu, orc):
    n, psi = I.dark_plane(3, 0.25, width=1.5)   # 64 x 6 x 6 intervals
    P = orc.Problem(3, n, 0.25, 0.5, -1.0, bc="msd")
    dt = 0.5 * P.max_dt(psi)
    say(f"[case] msd 3d dark plane n={n}")
    out, sol = gpu_run(gpu, 3, n, 0.25, psi, "f64", 30, dt)
    ref = P.rk4(psi, 30, dt)
    assert rel(out, ref) <= 1e-12
    assert line_err(out, ref) <= 1e-12
    sol.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_msd_variants_bit_identical(gpu, dim):
    g, psi = vortex_case(130) if dim == 2 else ring_case(36)
    sol = gpu.Solver(dim, g.n, g.h, 0.5, -1.0, None, "msd", "f64")
    nv = sol.variant_count()
    n_stage = 3 if dim == 2 else 4
    assert nv == (n_stage + 7 if dim == 2 else n_stage)   # 2D: the whole-step kernels run MSD too
    sol.set_field(psi)
    dt = 0.4 * sol.max_dt()
    sol.close()
    outs = []
    for v in range(nv):
        say(f"[case] msd {dim}d variant {v}")
        out, s2 = gpu_run(gpu, dim, g.n, g.h, psi, "f64", 5, dt, variant=v)
        assert s2.launches_per_step() == (8 if v < n_stage else 1)
        outs.append(out)
        s2.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


EPS = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "mixed": 2.0 ** -24}


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("case", ["vortex", "plane", "thin"])
def test_msd_whole_step_against_stage_path(gpu, orc, prec, case):
    """The 2D whole-step kernels under MSD (face values and boundary nodes formed inside the kernel,
    row 0 handed on one row late, row ny one row early).  Every segment length gives the same bits;
    against the MSD stage kernels the fields agree to the last place except for rare one-unit
    differences of the last place that start on the face y = 0 (in FP64 about one in 10^4 of its
    node-steps, more often in FP32) and spread over later steps; all match the oracle.  Grids: 131^2 (three strips, several segments), 128 x 64 nodes (ragged strips and
    segments), 128 x 5 nodes (every face row in the first groups)."""
    if case == "vortex":
        g, psi = vortex_case(130)
        n, h = g.n, g.h
    else:
        h = 0.125
        n, psi = I.dark_plane(2, h, lo=-8.0, hi=7.875, width=7.875 if case == "plane" else 0.5)
        rng = np.random.default_rng(5)
        psi = psi + 1e-3 * (rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))
    P = orc.Problem(2, n, h, 0.5, -1.0, bc="msd")
    dt = 0.5 * P.max_dt(psi)
    nst = 12
    sol = gpu.Solver(2, n, h, 0.5, -1.0, None, "msd", prec)
    nv = sol.variant_count()
    sol.close()
    assert nv == 10
    outs = []
    for v in [0] + list(range(3, nv)):
        say(f"[case] msd 2d whole step {case} n={n} {prec} variant {v}")
        out, s2 = gpu_run(gpu, 2, n, h, psi, prec, nst, dt, variant=v)
        assert s2.launches_per_step() == (8 if v == 0 else 1)
        s2.close()
        outs.append(np.asarray(out, np.complex128))
    for v, o in zip(range(4, nv), outs[2:]):
        assert np.array_equal(o, outs[1]), v            # segment lengths: the same bits
    d = np.abs(outs[1] - outs[0])
    scale = np.abs(outs[0]).max()
    say(f"[result] {case} {prec}: nodes differing from the stage path {int((d > 0).sum())}, max {d.max():.2e}")
    assert d[1:].max() <= 8 * EPS[prec] * scale             # rows 1 .. ny: at most rare last-place
    assert d[0].max() <= 8 * EPS[prec] * scale              # and row 0 likewise
    ref = P.rk4(psi, nst, dt)
    assert rel(outs[1], ref) <= TOL[prec]
    assert line_err(outs[1], ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64"])
def test_msd_whole_step_three_steps_bitwise(gpu, prec):
    """Over three FP64 steps the whole-step kernel under MSD gives the MSD stage kernels' bits (in FP32
    the rare last-place differences of the face y = 0 already show within three steps)."""
    g, psi = vortex_case(130)
    dt = None
    outs = []
    for v in (0, 3, 9):
        sol = gpu.Solver(2, g.n, g.h, 0.5, -1.0, None, "msd", prec)
        sol.set_field(psi.astype(sol.dtype))
        if dt is None:
            dt = 0.5 * sol.max_dt()
        sol.variant = v
        sol.step(3, dt)
        outs.append(sol.get_field())
        sol.close()
    assert np.array_equal(outs[1], outs[0]) and np.array_equal(outs[2], outs[0])


@pytest.mark.parametrize("dim", [2, 3])
def test_msd_bound_energy_mass(gpu, orc, dim):
    """The bound's boundary term, the energy (with the MSD step-1 face values of the current
    field) and the mass against the oracle."""
    g, psi = vortex_case(100) if dim == 2 else ring_case(30)
    P = orc.Problem(dim, g.n, g.h, 0.5, -1.0, bc="msd")
    say(f"[case] msd {dim}d bound/energy/mass n={g.n}")
    sol = gpu.Solver(dim, g.n, g.h, 0.5, -1.0, None, "msd", "f64")
    sol.set_field(psi)
    k, aux = P.max_dt(psi, return_aux=True)
    assert aux[2] > 0
    assert sol.max_dt() == pytest.approx(k, rel=1e-12)
    assert sol.energy() == pytest.approx(P.energy(psi), rel=1e-12)
    assert sol.mass() == pytest.approx(P.mass(psi), rel=1e-13)
    sol.close()


def test_msd_2d_batch_rejected(gpu):
    g, psi = vortex_case(64)
    spec = I.ProblemSpec("v", g, 0.5, -1.0, None, psi, "msd")
    with pytest.raises(gpu.NLSEError) as e:
        gpu.Batch([spec], prec="f32")
    assert e.value.code == -6


def test_msd_autotune_not_shared_with_dirichlet(gpu):
    """A Dirichlet context of the same shape tunes first; the MSD context must tune on its own
    (its whole-step kernels are other kernels) and keep its boundary rule."""
    g, psi = vortex_case(96)
    d = gpu.Solver(2, g.n, g.h, 0.5, -1.0, None, "dirichlet", "f32")
    d.set_field(psi.astype(np.complex64))
    d.autotune(reps=2, force=True)
    d.close()
    m = gpu.Solver(2, g.n, g.h, 0.5, -1.0, None, "msd", "f32")
    m.set_field(psi.astype(np.complex64))
    v = m.autotune(reps=2)
    assert 0 <= v < m.variant_count() and m.launches_per_step() == (8 if v < 3 else 1)
    m.close()


@pytest.mark.parametrize("dim,prec", [(2, "f64"), (2, "mixed"), (3, "f32")])
def test_msd_with_potential(gpu, orc, dim, prec):
    """MSD with V != 0: the N_{b-1} - N_b term of Eq. msdbc_lap and the V in F_{b-1} both enter."""
    g, psi = vortex_case(120) if dim == 2 else ring_case(32)
    c = g.coords()
    V = 0.02 * (c[0] + 0.5) ** 2 + 0.01 * c[1] + (0.005 * c[2] ** 2 if dim == 3 else 0.0)
    P = orc.Problem(dim, g.n, g.h, 0.5, -1.0, V=V, bc="msd")
    dt = 0.5 * P.max_dt(psi)
    nst = 30 if dim == 2 else 8
    say(f"[case] msd {dim}d with V, {prec}, {nst} steps")
    sol = gpu.Solver(dim, g.n, g.h, 0.5, -1.0, V, "msd", prec)
    sol.set_field(psi.astype(sol.dtype))
    assert sol.max_dt() == pytest.approx(P.max_dt(psi), rel=1e-4 if prec != "f64" else 1e-12)
    sol.step(nst, dt)
    out = sol.get_field()
    sol.close()
    ref = P.rk4(psi, nst, dt)
    assert rel(out, ref) <= TOL[prec]
    assert line_err(out, ref) <= TOL[prec]


def _case(dim):
    if dim == 1:
        n, psi = I.dark_plane(1, 0.125, lo=-8.0, hi=8.0, x0=-7.0)
        rng = np.random.default_rng(3)
        psi = psi + 1e-2 * (rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))
        return n[0], 0.125, psi
    g, psi = vortex_case(90) if dim == 2 else ring_case(30)
    return g.n, g.h, psi


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_msd_tiny_field(gpu, orc, dim, prec):
    """The whole field scaled by 1e-20 with s = 0 (linear, so the solution scales exactly).
    |Psi_{b-1}|^2 ~ 1e-40 is subnormal in FP32: the ratios Re(D_{b-1}/Psi_{b-1}) and
    Im(F_{b-1}/Psi_{b-1}) of Eqs. msdbc_lap / msdbc_ut must still come out right (the kernels
    scale numerator and denominator by a power of two before dividing)."""
    n, h, psi = _case(dim)
    psi = 1e-20 * psi
    P = orc.Problem(dim, n, h, 0.5, 0.0, bc="msd")
    dt = 0.5 * P.max_dt(psi)
    nst = 20 if dim < 3 else 6
    say(f"[case] msd {dim}d tiny field (|Psi| ~ 1e-20), s = 0, {prec}, {nst} steps")
    sol = gpu.Solver(dim, n, h, 0.5, 0.0, None, "msd", prec)
    sol.set_field(psi.astype(sol.dtype))
    sol.step(nst, dt)
    out = sol.get_field()
    sol.close()
    ref = P.rk4(psi, nst, dt)
    e = rel(out, ref)
    say(f"[result] msd {dim}d tiny field {prec}: rel L2 {e:.3e}")
    assert np.isfinite(out).all()
    assert e <= TOL[prec]
    assert line_err(out, ref) <= TOL[prec]


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_msd_zero_b_minus_1(gpu, orc, dim, prec):
    """Psi_{b-1} = 0 at some boundary neighbours (reading: the ratio term of Eq. msdbc_lap and the
    phase rate of Eq. msdbc_ut are dropped there): GPU against the oracle."""
    n, h, psi = _case(dim)
    psi = psi.copy()
    if dim == 1:
        psi[1] = 0.0
        psi[-2] = 0.0
    elif dim == 2:
        psi[10:30, 1] = 0.0          # the x = 0 face's inner neighbours
        psi[-2, 40:60] = 0.0         # the y = ny face's
        psi[1, 1] = 0.0              # the corner's diagonal neighbour
    else:
        psi[5:12, 5:12, 1] = 0.0
        psi[1, 8:20, 8:20] = 0.0
    P = orc.Problem(dim, n, h, 0.5, -1.0, bc="msd")
    dt = 0.5 * P.max_dt(psi)
    nst = 12 if dim < 3 else 4
    say(f"[case] msd {dim}d with Psi_(b-1) = 0 on part of the boundary, {prec}, {nst} steps")
    sol = gpu.Solver(dim, n, h, 0.5, -1.0, None, "msd", prec)
    sol.set_field(psi.astype(sol.dtype))
    sol.step(nst, dt)
    out = sol.get_field()
    sol.close()
    ref = P.rk4(psi, nst, dt)
    e = rel(out, ref)
    say(f"[result] msd {dim}d zero b-1 {prec}: rel L2 {e:.3e}")
    assert np.isfinite(out).all()
    assert e <= TOL[prec]
    assert line_err(out, ref) <= TOL[prec]
