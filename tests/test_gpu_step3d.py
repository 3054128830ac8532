"""The 3D two-stage kernels (stages 1+2 and 3+4 fused, two launches per RK4 step).

They evaluate every point with the stage kernels' point-wise code, so their fields must be
bitwise equal to four stage launches for every variant, precision, grid shape (non-cubic,
ragged tiles, grids smaller than one tile), odd step counts (the master buffers swap) and
non-zero Dirichlet values; and they meet the oracle at the parity tolerances.
"""
import sys

import numpy as np
import pytest

import nlse_inputs as I

pytestmark = pytest.mark.gpu


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


def pair_variants(s):
    out = []
    for v in range(s.variant_count()):
        s.variant = v
        if s.launches_per_step() == 2:
            out.append(v)
    s.variant = 0
    return out


def run(gpu, n, h, psi, V, prec, variant, steps, dt):
    s = gpu.Solver(3, n, h, 0.5, -1.0, V, "dirichlet", prec)
    s.set_field(psi.astype(s.dtype))
    s.variant = variant
    s.step(steps, dt)
    out = s.get_field()
    s.close()
    return out


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("n", [(70, 70, 70), (61, 23, 9), (5, 4, 6), (130, 17, 40), (2, 2, 2), (3, 2, 5)])
def test_pairs_bitwise_equal_to_stage_kernels(gpu, prec, n):
    psi, V = I.smooth_random_3d(n, 3, boundary_amp=0.3)
    h = 1.0 / max(n)
    s = gpu.Solver(3, n, h, 0.5, -1.0, V, "dirichlet", prec)
    s.set_field(psi.astype(s.dtype))
    dt = 0.4 * s.max_dt()
    pv = pair_variants(s)
    s.close()
    assert len(pv) == 3
    ref = run(gpu, n, h, psi, V, prec, 0, 5, dt)
    for v in pv:
        say(f"[case] 3D pairs variant {v} {prec} n={n}, 5 steps")
        got = run(gpu, n, h, psi, V, prec, v, 5, dt)
        assert np.array_equal(got, ref), (v, float(np.max(np.abs(got - ref))))


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
def test_pairs_oracle_parity(gpu, orc, prec):
    sp = I.config_gp3d(n=70)
    P = orc.Problem.from_spec(sp)
    dt = 0.5 * P.max_dt(sp.psi0)
    ref = P.rk4(sp.psi0, 7, dt)
    s = gpu.Solver.from_spec(sp, prec=prec)
    s.set_field(sp.psi0)
    v = pair_variants(s)[0]
    s.variant = v
    say(f"[case] 3D GP n=70 {prec} pair variant {v}, 7 steps vs oracle")
    s.step(7, dt)
    g = np.asarray(s.get_field(), np.complex128)
    s.close()
    e = float(np.linalg.norm((g - ref).ravel()) / np.linalg.norm(ref.ravel()))
    say(f"  rel L2 = {e:.3e}")
    assert e <= (1e-12 if prec == "f64" else 1e-4)


def test_pairs_mixed_with_stage_kernels(gpu):
    """Switching between pair and stage variants mid-run (the master buffers swap) changes nothing."""
    n = (66, 31, 20)
    psi, V = I.smooth_random_3d(n, 5)
    h = 1.0 / 66
    s = gpu.Solver(3, n, h, 0.5, -1.0, V, "dirichlet", "f32")
    s.set_field(psi.astype(np.complex64))
    dt = 0.4 * s.max_dt()
    pv = pair_variants(s)
    for v in (pv[0], 0, pv[1], pv[1], 2, pv[2], pv[0]):
        s.variant = v
        s.step(1, dt)
    got = s.get_field()
    s.close()
    ref = run(gpu, n, h, psi, V, "f32", 0, 7, dt)
    assert np.array_equal(got, ref)


def test_pairs_not_offered_under_msd(gpu):
    g = I.grid(3, 20, -8.0, 8.0)
    s = gpu.Solver(3, 20, g.h, 0.5, -1.0, None, "msd", "f32")
    assert pair_variants(s) == []
    s.close()
