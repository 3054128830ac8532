"""The 2D whole-step kernel (all four RK4 stages in one launch) on the GPU.

It performs the same floating-point operations as the four stage launches, so it is checked
bit for bit against them, and against the FP64 oracle at the parity tolerances (FP64 <= 1e-12,
FP32 / mixed <= 1e-4 relative L2).  Sizes cover one strip, several 48-column strips and row
segments with ragged tails, grids with inner tasks (no boundary node within a wave's reach,
the code path without face closures) beside boundary tasks, non-square grids, odd step
counts (the master buffers swap every step) and switches between kernel kinds in the middle
of a run.
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


def whole_step_variants(s):
    """Variants whose RK4 step is one launch."""
    out = []
    for v in range(s.variant_count()):
        s.variant = v
        if s.launches_per_step() == 1:
            out.append(v)
    s.variant = 0
    return out


def gp2d_problem(nx, ny, seed=2, boundary=False):
    """The 2D GP workload on an nx x ny-interval grid over [-40, 40] x [-40*ny/nx, ...] (h fixed)."""
    h = 80.0 / nx
    x = -40.0 + h * np.arange(nx + 1)
    y = -(h * ny) / 2 + h * np.arange(ny + 1)
    X, Y = np.meshgrid(x, y)
    V = 0.5 * 0.05 ** 2 * (X ** 2 + Y ** 2)
    rng = np.random.default_rng(seed)
    r = np.hypot(X, Y)
    psi = np.sqrt(np.maximum(1.0 - V, 0.0)) * np.tanh(r) * np.exp(1j * np.arctan2(Y, X))
    psi = psi + 1e-3 * (rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))
    m = np.zeros(psi.shape, bool)
    m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = True
    psi[m] = 0.3 * (rng.standard_normal(m.sum()) + 1j * rng.standard_normal(m.sum())) if boundary else 0.0
    return h, V, psi


def run(gpu, nx, ny, prec, variant, steps, h, V, psi, dt=None, V_on=True):
    s = gpu.Solver(2, (nx, ny), h, 0.5, -1.0, V if V_on else None, prec=prec)
    s.set_field(psi)
    if dt is None:
        dt = min(0.5 * s.max_dt(), 0.05)   # the cap keeps the coarsest grids (h = 40) finite
    s.variant = variant
    s.step(steps, dt)
    return s.get_field(), s, dt


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("nx,ny", [(2, 2), (5, 7), (49, 30), (150, 97), (97, 150), (200, 64), (300, 260)])
def test_whole_step_bitwise_equals_stage_kernels(gpu, prec, nx, ny):
    h, V, psi = gp2d_problem(nx, ny, boundary=True)
    ref, s, dt = run(gpu, nx, ny, prec, 0, 7, h, V, psi)
    assert np.isfinite(ref).all()
    for v in whole_step_variants(s):
        say(f"[case] whole-step variant {v} {prec} {nx}x{ny}, 7 steps")
        got, _, _ = run(gpu, nx, ny, prec, v, 7, h, V, psi, dt)
        assert np.array_equal(got, ref), (v, rel(got, ref))


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("n", [5, 70, 150])
def test_whole_step_parity_with_oracle(gpu, orc, prec, n):
    sp = I.config_gp2d(n=n)
    P = orc.Problem.from_spec(sp)
    dt = 0.5 * P.max_dt(sp.psi0)
    ref = P.rk4(sp.psi0, 30, dt)
    s = gpu.Solver.from_spec(sp, prec=prec)
    s.set_field(sp.psi0)
    for v in whole_step_variants(s):
        say(f"[case] config_gp2d n={n} {prec} whole-step variant {v}, 30 steps")
        s.set_field(sp.psi0)
        s.variant = v
        s.step(30, dt)
        got = s.get_field()
        e = rel(got, ref)
        say(f"[result] rel L2 {e:.3e}")
        assert e <= TOL[prec], (v, e)
        assert line_err(got, ref) <= TOL[prec]


def test_whole_step_no_potential_and_fixed_boundary(gpu, orc):
    nx, ny = 131, 77
    h, V, psi = gp2d_problem(nx, ny, seed=9, boundary=True)
    P = orc.Problem(2, (nx, ny), h, 0.5, -1.0, None)
    dt = 0.5 * P.max_dt(psi)
    ref = P.rk4(psi, 11, dt)
    s = gpu.Solver(2, (nx, ny), h, 0.5, -1.0, None, prec="f64")
    for v in whole_step_variants(s):
        s.set_field(psi)
        s.variant = v
        s.step(11, dt)
        g = s.get_field()
        assert rel(g, ref) <= 1e-12
        assert line_err(g, ref) <= 1e-12
        m = np.zeros(psi.shape, bool)
        m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = True
        assert np.array_equal(g[m], psi[m]), "Dirichlet values must stay fixed"


def test_switching_kernel_kinds_mid_run(gpu):
    nx, ny = 150, 120
    h, V, psi = gp2d_problem(nx, ny)
    ref, s, dt = run(gpu, nx, ny, "f64", 0, 10, h, V, psi)
    ws = whole_step_variants(s)
    s = gpu.Solver(2, (nx, ny), h, 0.5, -1.0, V, prec="f64")
    s.set_field(psi)
    plan = [(ws[0], 3), (1, 2), (ws[-1], 1), (2, 1), (ws[1], 3)]
    for v, k in plan:
        s.variant = v
        s.step(k, dt)
    assert np.array_equal(s.get_field(), ref)
    m0 = s.mass()
    r = gpu.Solver(2, (nx, ny), h, 0.5, -1.0, V, prec="f64")
    r.set_field(ref)
    assert m0 == r.mass()


def test_set_field_after_odd_steps(gpu):
    """After an odd number of whole steps the master buffers have swapped; a new field and
    further steps must behave exactly as on a fresh context."""
    nx, ny = 90, 90
    h, V, psi = gp2d_problem(nx, ny, seed=3)
    _, _, psi2 = gp2d_problem(nx, ny, seed=4, boundary=True)
    ref, s0, dt = run(gpu, nx, ny, "f32", 0, 5, h, V, psi2)
    s = gpu.Solver(2, (nx, ny), h, 0.5, -1.0, V, prec="f32")
    s.set_field(psi)
    s.variant = whole_step_variants(s)[0]
    s.step(3, dt)
    s.set_field(psi2)
    s.step(5, dt)
    assert np.array_equal(s.get_field(), ref)


def test_whole_step_full_size(gpu, orc):
    """The benchmark's workload (2049^2 nodes), two steps of every whole-step variant."""
    sp = I.config_gp2d(n=2048)
    P = orc.Problem.from_spec(sp)
    dt = 0.5 * P.max_dt(sp.psi0)
    ref = P.rk4(sp.psi0, 2, dt)
    for prec in ("f64", "f32", "mixed"):
        s = gpu.Solver.from_spec(sp, prec=prec)
        for v in whole_step_variants(s):
            say(f"[case] 2049^2 {prec} whole-step variant {v}, 2 steps")
            s.set_field(sp.psi0)
            s.variant = v
            s.step(2, dt)
            got = s.get_field()
            e = rel(got, ref)
            say(f"[result] rel L2 {e:.3e}")
            assert e <= TOL[prec], (prec, v, e)
            assert line_err(got, ref) <= TOL[prec]
        s.close()
