"""nlse_mass_noalloc (the entry point for callers that cannot allocate) against nlse_mass.

Both reduce h^d sum |Psi|^2 in FP64 in the same fixed order (rows to blocks, then a fixed
tree), so the values must agree bit for bit.  Two calls in a row on one GPU share the
library's static scratch; the second uses a smaller field, so stale partial sums of the
first would show."""
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


def _field(dim, n, seed):
    rng = np.random.default_rng(seed)
    shape = (n + 1,) * dim if np.isscalar(n) else tuple(int(k) + 1 for k in reversed(n))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _ctx_mass(P, dim, n, h, prec, psi):
    s = P.Solver(dim, n, h, 0.5, -1.0, None, "dirichlet", prec)
    s.set_field(psi.astype(s.dtype))
    m = s.mass()
    s.close()
    return m


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
def test_mass_noalloc_matches_ctx_mass_two_calls(gpu, prec):
    import torch
    cases = [(2, 300, 0.07, 1), (2, 37, 0.3, 2), (3, (20, 11, 7), 0.2, 3), (1, 50, 0.5, 4)]
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for dim, n, h, seed in cases:          # each call smaller than the one before
        psi = _field(dim, n, seed)
        want = _ctx_mass(gpu, dim, n, h, prec, psi)
        dt = torch.complex64 if prec == "f32" else torch.complex128
        t = torch.from_numpy(psi).to(dt).cuda()
        say(f"[case] mass_noalloc {prec} dim={dim} n={n}")
        gpu.mass_noalloc(t, h, prec, out)
        torch.cuda.synchronize()
        got = float(out.item())
        say(f"[result] mass_noalloc {prec} dim={dim} n={n}: {got!r} vs nlse_mass {want!r}")
        assert got == want


def test_mass_noalloc_rejects_bad_arguments(gpu):
    import torch
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = torch.zeros((5, 5), dtype=torch.complex128, device="cuda")
    with pytest.raises(gpu.NLSEError):
        gpu.mass_noalloc(t, -1.0, "f64", out)
    with pytest.raises(gpu.NLSEError):
        gpu.mass_noalloc(t, float("inf"), "f64", out)
    one = torch.zeros((1,), dtype=torch.complex128, device="cuda")   # n = 0 intervals
    with pytest.raises(gpu.NLSEError):
        gpu.mass_noalloc(one, 1.0, "f64", out)
