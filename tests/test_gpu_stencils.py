"""The alternative 1D, 2D and 3D Laplacians (nlse_set_stencil) against the oracle.

The non-compact fourth-order stencil and the second-order CD are what 2SHOC is compared with
(Sec. 2.1, Sec. 5).  The oracle implements both (lap="noncompact", whose ghost one node beyond
a boundary node b is 2 Psi_b - Psi_{b+-1} + h^2 D^a_b with D^a_b the step-1 face value of
Eq. dbc_lap; lap="cd"); parity bars as for 2SHOC: FP64 <= 1e-12, FP32 <= 1e-4 relative L2.
Non-zero Dirichlet values make the ghosts matter.
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


def with_random_boundary(spec, seed=5, amp=0.3):
    rng = np.random.default_rng(seed)
    psi = spec.psi0.copy()
    m = spec.grid.boundary_mask()
    psi[m] = amp * (rng.standard_normal(m.sum()) + 1j * rng.standard_normal(m.sum()))
    return I.ProblemSpec(spec.name + "_bnd", spec.grid, spec.a, spec.s, spec.V, psi, spec.bc)


@pytest.mark.parametrize("stencil", ["noncompact", "cd"])
@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("n,boundary", [(5, False), (70, True), (150, True)])
def test_stencil_parity_with_oracle(gpu, orc, stencil, prec, n, boundary):
    """2D alternative Laplacians against the oracle, in the stage kernels (variant 0) and in the
    whole-step kernel (the last variant)."""
    sp = I.config_gp2d(n=n)
    if boundary:
        sp = with_random_boundary(sp)
    P = orc.Problem.from_spec(sp, lap=stencil)
    dt = 0.5 * orc.Problem.from_spec(sp).max_dt(sp.psi0)
    ref = P.rk4(sp.psi0, 20, dt)
    s = gpu.Solver.from_spec(sp, prec=prec)
    s.stencil = stencil
    assert s.stencil == stencil
    for v in (0, s.variant_count() - 1):
        s.variant = v
        s.set_field(sp.psi0)
        s.step(20, dt)
        got = s.get_field()
        e = rel(got, ref)
        say(f"[result] {stencil} {prec} n={n} variant {v}: rel L2 {e:.3e}")
        assert e <= TOL[prec]
        assert line_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("stencil", ["noncompact", "cd"])
@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("nx,ny", [(150, 150), (300, 260), (97, 41)])
def test_stencil_variants_bitwise_and_api(gpu, stencil, prec, nx, ny):
    """2D: the stage kernels and the whole-step kernels (every segment length) evaluate the
    alternative Laplacians with the same operations, so all variants give the same bits
    (random Dirichlet values, grids with inner and boundary tasks, ragged strips)."""
    h = 80.0 / max(nx, ny)
    x = -40.0 + h * np.arange(nx + 1)
    y = -(h * ny) / 2 + h * np.arange(ny + 1)
    X, Y = np.meshgrid(x, y)
    V = 0.5 * 0.05 ** 2 * (X ** 2 + Y ** 2)
    rng = np.random.default_rng(nx + ny)
    psi = np.sqrt(np.maximum(1.0 - V, 0.0)) * np.tanh(np.hypot(X, Y)) * np.exp(1j * np.arctan2(Y, X))
    psi = psi + 1e-3 * (rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))
    m = np.zeros(psi.shape, bool)
    m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = True
    psi[m] = 0.3 * (rng.standard_normal(m.sum()) + 1j * rng.standard_normal(m.sum()))
    s0 = gpu.Solver(2, (nx, ny), h, 0.5, -1.0, V, prec=prec)
    n_all = s0.variant_count()
    s0.stencil = stencil
    assert s0.variant_count() == n_all     # the whole-step variants stay for every 2D stencil
    s0.set_field(psi.astype(s0.dtype))
    dt = 0.5 * s0.max_dt()
    s0.close()
    outs = []
    for v in range(n_all):
        s = gpu.Solver(2, (nx, ny), h, 0.5, -1.0, V, prec=prec)
        s.stencil = stencil
        s.set_field(psi.astype(s.dtype))
        s.variant = v
        say(f"[case] 2D {stencil} {prec} {nx}x{ny} variant {v} ({s.launches_per_step()} launches per step), 7 steps")
        s.step(7, dt)
        outs.append(s.get_field())
        s.close()
    for v, o in enumerate(outs[1:], 1):
        assert np.array_equal(o, outs[0]), v


@pytest.mark.parametrize("stencil", ["noncompact", "cd"])
@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("n", [(5, 5, 5), (40, 40, 40), (61, 23, 9), (70, 18, 33), (2, 3, 2)])
def test_stencil3d_parity_with_oracle(gpu, orc, stencil, prec, n):
    """3D stage kernels: 13-point non-compact cross and 7-point CD, random Dirichlet values,
    ragged tiles in every direction, grids smaller than a tile."""
    psi, V = I.smooth_random_3d(n, 7, boundary_amp=0.3)
    h = 1.0 / max(n)
    dt = 0.4 * orc.Problem(3, n, h, 0.5, -1.0, V).max_dt(psi)
    ref = orc.Problem(3, n, h, 0.5, -1.0, V, lap=stencil).rk4(psi, 10, dt)
    s = gpu.Solver(3, n, h, 0.5, -1.0, V, "dirichlet", prec)
    s.stencil = stencil
    s.set_field(psi.astype(s.dtype))
    say(f"[case] 3D {stencil} {prec} n={n}, 10 steps")
    s.step(10, dt)
    got = s.get_field()
    e = rel(got, ref)
    s.close()
    say(f"[result] 3D {stencil} {prec} n={n}: rel L2 {e:.3e}")
    assert e <= TOL[prec]
    assert line_err(got, ref) <= TOL[prec]


@pytest.mark.parametrize("stencil", ["noncompact", "cd"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_stencil3d_variants_bitwise_and_api(gpu, stencil, prec):
    n = (66, 37, 70)
    psi, V = I.smooth_random_3d(n, 9, boundary_amp=0.3)
    h = 1.0 / 70
    s0 = gpu.Solver(3, n, h, 0.5, -1.0, V, "dirichlet", prec)
    n_all = s0.variant_count()
    s0.variant = n_all - 1                 # a two-stage variant
    s0.stencil = stencil
    assert s0.variant == 0 and s0.variant_count() == 4
    with pytest.raises(gpu.NLSEError):
        s0.variant = 4
    s0.stencil = "2shoc"
    assert s0.variant_count() == n_all
    s0.close()
    outs = []
    for v in range(4):
        s = gpu.Solver(3, n, h, 0.5, -1.0, V, "dirichlet", prec)
        s.stencil = stencil
        s.set_field(psi.astype(s.dtype))
        s.variant = v
        assert s.launches_per_step() == 4
        say(f"[case] 3D {stencil} {prec} variant {v}, 5 steps")
        s.step(5, 0.4 * s.max_dt())
        outs.append(s.get_field())
        s.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("stencil", ["noncompact", "cd"])
@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("n", [2, 3, 5, 1024, 5119])
def test_stencil1d_parity_with_oracle(gpu, orc, stencil, prec, n):
    """The on-chip 1D solver with the five-point non-compact stencil (two nodes of each
    neighbouring thread, ghosts carrying the face value) and with CD, random Dirichlet values; every
    variant that holds the field gives the same bits."""
    if prec == "f64" and n + 1 > 5120:
        pytest.skip("beyond the FP64 on-chip capacity")
    rng = np.random.default_rng(n)
    g = I.grid(1, n, -10, 10)
    (x,) = g.coords()
    psi = I.bright_soliton(x, 0.0, 1.0, 1.0, 1.2, 0.3).astype(np.complex128)
    psi[0], psi[-1] = 0.3 * (rng.standard_normal(2) + 1j * rng.standard_normal(2))
    V = 0.05 * x * x
    sp = I.ProblemSpec("st1d", g, 1.0, 1.0, V, psi, "dirichlet")
    # On the tiniest grids the bound of Eq. kdfull is not a stability guarantee (it is the
    # large-n limit): with n = 3 and these boundary values both fourth-order stencils blow up
    # at 0.3 x the bound in the oracle, so those grids take a smaller step.
    dt = (0.5 if n >= 8 else 0.2) * orc.Problem.from_spec(sp).max_dt(psi)
    ref = orc.Problem.from_spec(sp, lap=stencil).rk4(psi, 30, dt)
    assert np.isfinite(ref).all()
    outs = []
    s0 = gpu.Solver.from_spec(sp, prec=prec)
    nv = s0.variant_count()
    s0.close()
    for v in range(nv):
        s = gpu.Solver.from_spec(sp, prec=prec)
        s.stencil = stencil
        s.variant = v
        s.set_field(psi.astype(s.dtype))
        say(f"[case] 1D {stencil} {prec} n={n} variant {v}")
        s.step(30, dt)
        outs.append(s.get_field())
        s.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    e = rel(outs[0], ref)
    say(f"[result] 1D {stencil} {prec} n={n}: rel L2 {e:.3e}")
    assert e <= TOL[prec]
    assert line_err(outs[0], ref) <= TOL[prec]


@pytest.mark.parametrize("dim,n", [(1, 300), (2, 90), (3, (37, 21, 30))])
def test_noncompact_equals_2shoc_any_dirichlet(gpu, dim, n):
    """Sec. 2.1: the two-step scheme is the five-point fourth-order stencil.  With the ghost that
    carries the face value, the GPU's non-compact runs equal its 2SHOC runs to round-off for
    random non-zero Dirichlet values as well (FP64, 20 steps)."""
    rng = np.random.default_rng(11 + dim)
    if dim == 3:
        psi, V = I.smooth_random_3d(n, 3, boundary_amp=0.3)
        h = 1.0 / max(n)
        args = (3, n, h, 0.5, -1.0, V)
    else:
        g = I.grid(dim, n, -6.0, 6.0)
        sp = I.config_gp2d(n=n) if dim == 2 else None
        if dim == 2:
            psi, V = sp.psi0.copy(), sp.V
            args = (2, n, sp.grid.h, sp.a, sp.s, V)
        else:
            (x,) = g.coords()
            psi = I.bright_soliton(x, 0.0, 1.0, 1.0, 1.2, 0.3).astype(np.complex128)
            V = 0.05 * x * x
            args = (1, n, g.h, 1.0, 1.0, V)
        m = np.zeros(psi.shape, bool)
        for ax in range(dim):
            idx = [slice(None)] * dim
            idx[ax] = 0
            m[tuple(idx)] = True
            idx[ax] = -1
            m[tuple(idx)] = True
        psi[m] = 0.3 * (rng.standard_normal(m.sum()) + 1j * rng.standard_normal(m.sum()))
    outs = []
    for stencil in ("2shoc", "noncompact"):
        s = gpu.Solver(*args, "dirichlet", "f64")
        s.stencil = stencil
        s.set_field(psi)
        dt = 0.4 * s.max_dt()
        say(f"[case] {dim}D {stencil} f64 n={n}, 20 steps, random Dirichlet values")
        s.step(20, dt)
        outs.append(s.get_field())
        s.close()
    e = rel(outs[1], outs[0])
    say(f"[result] {dim}D noncompact vs 2shoc: rel L2 {e:.3e}")
    assert e <= 1e-12


def test_stencil_unsupported_under_msd(gpu):
    for dim in (1, 2, 3):
        g = I.grid(dim, 20, -8.0, 8.0)
        s = gpu.Solver(dim, 20, g.h, 0.5, -1.0, None, "msd", "f32")
        for name in ("noncompact", "cd"):
            with pytest.raises(gpu.NLSEError):
                s.stencil = name
        assert s.stencil == "2shoc"
        s.close()
