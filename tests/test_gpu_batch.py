"""Batched persistent launch: per-instance parity with the FP64 oracle, bitwise agreement
with single-instance contexts, and the full batched workload (4096 1D + 256 2D instances)
checked on a sample of instances covering min/max size, both signs of s and the extremes
of the trap frequency."""
import sys

import numpy as np
import pytest

import nlse_inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available()
    import paper_1109_1027_amd as P
    P.load()
    return P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a, np.complex128) - b).ravel()) / np.linalg.norm(b.ravel()))


def small_mix(seed=7):
    """A small uneven mix: 1D bright (Dirichlet) and dark (MSD) at the size extremes, 2D GP."""
    specs = I.batch_instances(n1d=12, n2d=3, seed=seed, n2d_grid=96)
    g = I.grid(1, 256, -16, 16)
    (x,) = g.coords()
    specs.append(I.ProblemSpec("dark256", g, 1.0, -1.0, None, I.dark_soliton(x, 0.0, omega=-2.0, c=0.3), "msd"))
    g = I.grid(1, 8192, -512, 512)
    (x,) = g.coords()
    b = I.bright_soliton(x, 0.0, 1.0, 1.0, 1.0, 0.2)
    b[0] = b[-1] = 0
    specs.append(I.ProblemSpec("bright8192", g, 1.0, 1.0, None, b, "dirichlet"))
    return specs


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_matches_oracle(gpu, orc, prec):
    specs = small_mix()
    if prec == "f64":
        specs = [sp for sp in specs if sp.grid.n + 1 <= 5120]
    say(f"[case] batch of {len(specs)} instances, {prec}, 60 steps")
    b = gpu.Batch(specs, prec=prec)
    b.set_fields(specs)
    dts = b.set_dts(0.5)
    b.step(60)
    b.sync()
    tol = 1e-4 if prec == "f32" else 1e-12
    for i, sp in enumerate(specs):
        ref = orc.Problem.from_spec(sp).rk4(sp.psi0, 60, dts[i])
        err = rel(b.get_field(i), ref)
        assert err <= tol, (sp.name, sp.grid.n, err)


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_batch_bitwise_equals_single(gpu, variant):
    specs = small_mix(seed=9)
    b = gpu.Batch(specs, prec="f32")
    b.set_fields(specs)
    dts = b.set_dts(0.5)
    b.variant = variant
    say(f"[case] batch vs single contexts, variant {variant}")
    b.step(25)
    for i, sp in enumerate(specs):
        s = gpu.Solver.from_spec(sp, prec="f32")
        s.set_field(sp.psi0)
        s.step(25, dts[i])
        assert np.array_equal(b.get_field(i), s.get_field()), sp.name


def test_batch_graph_replay_and_autotune(gpu):
    """Two 10-step graph replays equal one 20-step launch; autotuning restores the state."""
    specs = small_mix(seed=3)
    a = gpu.Batch(specs, prec="f32")
    a.set_fields(specs)
    a.set_dts(0.5)
    v = a.autotune(nsteps=5, force=True)
    assert 0 <= v < a.variant_count()
    a.step(10)
    a.step(10)
    c = gpu.Batch(specs, prec="f32")
    c.set_fields(specs)
    c.set_dts(0.5)
    c.variant = v
    c.step(20)
    for i in range(len(specs)):
        assert np.array_equal(a.get_field(i), c.get_field(i))


def test_batch_rejects_bad_input(gpu):
    specs = small_mix(seed=1)[:3]
    b = gpu.Batch(specs, prec="f32")
    with pytest.raises(gpu.NLSEError):
        b.step(1)                       # no fields / dts yet
    b.set_fields(specs)
    with pytest.raises(gpu.NLSEError) as e:
        b.set_dt(0, 2.0 * b.max_dt(0))
    assert e.value.code == -2
    with pytest.raises(gpu.NLSEError):
        b.set_dt(99, 0.1)


def test_batch_full_workload_sampled(gpu, orc):
    """The full batched workload (4096 1D n in [256, 8192] + 256 2D at 256^2, seed 4), 1000 steps
    in one graph launch; sampled instances against the oracle."""
    specs = I.batch_instances()
    say(f"[case] full batch: {len(specs)} instances, f32, 1000 steps")
    b = gpu.Batch(specs, prec="f32")
    b.set_fields(specs)
    dts = b.set_dts(0.5)
    b.autotune(nsteps=5)
    b.step(1000)
    b.sync()
    ones = [i for i, sp in enumerate(specs) if sp.dim == 1]
    twos = [i for i, sp in enumerate(specs) if sp.dim == 2]
    ns = [specs[i].grid.n for i in ones]
    pick = {ones[int(np.argmin(ns))], ones[int(np.argmax(ns))]}
    pick |= {next(i for i in ones if specs[i].s > 0), next(i for i in ones if specs[i].s < 0)}
    oms = [specs[i].grid.hi for i in twos]          # half-width 2/omega: extremes of omega
    pick |= {twos[int(np.argmin(oms))], twos[int(np.argmax(oms))]}
    for i in sorted(pick):
        sp = specs[i]
        ref = orc.Problem.from_spec(sp).rk4(sp.psi0, 1000, dts[i])
        err = rel(b.get_field(i), ref)
        say(f"[result] instance {i} {sp.name} n={sp.grid.n}: rel L2 {err:.2e}")
        assert err <= 1e-4, (sp.name, err)
