"""Learned corrector on the GPU (BF16 MFMA forward and backward) against the CPU reference
of oracle/conv.py, which emulates the same bf16 rounding points in FP64."""
import sys

import numpy as np
import pytest

import nlse_inputs as I
from oracle import conv

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


def flat(p):
    return np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)


def nontrivial_params(seed):
    rng = np.random.default_rng(seed)
    p = conv.init_params(seed)
    p["W3"] = (rng.standard_normal(p["W3"].shape) * 0.2).astype(np.float32).astype(np.float64)
    for b in ("b1", "b2", "b3"):
        p[b] = (rng.standard_normal(p[b].shape) * 0.1).astype(np.float32).astype(np.float64)
    return p


def fields(n=64, seeds=(1, 2)):
    g = I.grid(2, n, -40, 40)
    out = [I.gp2d_multivortex(g, seed=s) for s in seeds]
    return g, np.stack([o[0] for o in out]).astype(np.complex64), out[0][1]


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_forward_matches_cpu(gpu):
    import torch
    g, psi, V = fields()
    p = nontrivial_params(3)
    m = gpu.Corrector(g.nodes, g.nodes, max_batch=2, V=V)
    m.set_params(flat(p), 1.0)
    y = m.infer(torch.from_numpy(psi).cuda()).cpu().numpy()
    for b in range(2):
        ref, _ = conv.forward(p, conv.features(psi[b], V, g.h), emulate=True)
        err = rel(y[b], ref)
        say(f"[result] forward sample {b}: rel err {err:.2e}")
        assert err < 2e-3


def test_gradients_match_cpu(gpu):
    import torch
    g, psi, V = fields(n=48, seeds=(4, 5))
    rng = np.random.default_rng(9)
    ref_f = (psi + 0.01 * (rng.standard_normal(psi.shape) + 1j * rng.standard_normal(psi.shape))).astype(np.complex64)
    scale = 0.01
    p = nontrivial_params(7)
    m = gpu.Corrector(g.nodes, g.nodes, max_batch=2, V=V)
    m.set_params(flat(p), scale)
    loss, gr = m.grads(torch.from_numpy(psi).cuda(), torch.from_numpy(ref_f).cuda())
    tot, refg = 0.0, None
    for b in range(2):
        # the GPU forms (ref - pred) / scale in FP32
        T = (np.stack([(ref_f[b].real.astype(np.float32) - psi[b].real.astype(np.float32)),
                       (ref_f[b].imag.astype(np.float32) - psi[b].imag.astype(np.float32))], axis=-1)
             * np.float32(1.0 / scale)).astype(np.float64)
        l, gg, _ = conv.loss_and_grads(p, conv.features(psi[b], V, g.h), T, emulate=True)
        tot += l / 2
        gflat = flat({k: v / 2 for k, v in gg.items()}).astype(np.float64)
        refg = gflat if refg is None else refg + gflat
    assert loss == pytest.approx(tot, rel=2e-3)
    offs = {"W1": (0, 2304), "b1": (2304, 2336), "W2": (2336, 11552), "b2": (11552, 11584),
            "W3": (11584, 12160), "b3": (12160, 12162)}
    for k, (a, b) in offs.items():
        err = rel(gr[a:b].astype(np.float64), refg[a:b])
        say(f"[result] grad {k}: rel err {err:.2e}")
        assert err < 3e-2, k


def test_training_reduces_loss(gpu):
    import torch
    g, psi, V = fields(n=64, seeds=(11, 12))
    rng = np.random.default_rng(2)
    ref = (psi + 1e-3 * (psi * np.abs(psi))).astype(np.complex64)   # a smooth, learnable residual
    m = gpu.Corrector(g.nodes, g.nodes, max_batch=2, V=V)
    m.set_params(flat(conv.init_params(0)), 1e-3)
    tp, tr = torch.from_numpy(psi).cuda(), torch.from_numpy(ref).cuda()
    losses = [m.train_step(tp, tr, 3e-3) for _ in range(60)]
    say(f"[result] loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert losses[-1] < 0.5 * losses[0]


def test_apply_matches_infer(gpu):
    import torch
    g, psi, V = fields(n=64, seeds=(21,))
    p = nontrivial_params(1)
    m = gpu.Corrector(g.nodes, g.nodes, max_batch=1, V=V)
    m.set_params(flat(p), 0.01)
    s = gpu.Solver(2, g.n, g.h, 0.5, -1.0, V, prec="f32")
    s.set_field(psi[0])
    y = m.infer(torch.from_numpy(psi[0]).cuda()).cpu().numpy()[0]
    m.apply(s)
    out = s.get_field()
    want = psi[0].copy()
    want[1:-1, 1:-1] += (np.float32(0.01) * (y[1:-1, 1:-1, 0] + 1j * y[1:-1, 1:-1, 1])).astype(np.complex64)
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-6)
    assert np.array_equal(out[0], psi[0][0])


def test_inject(gpu):
    import torch
    rng = np.random.default_rng(0)
    src = (rng.standard_normal((257, 257)) + 1j * rng.standard_normal((257, 257))).astype(np.complex64)
    dst = torch.empty((65, 65), dtype=torch.complex64, device="cuda")
    gpu.inject(torch.from_numpy(src).cuda(), 256, dst, 4)
    assert np.array_equal(dst.cpu().numpy(), src[::4, ::4])
    src64 = src.astype(np.complex128)
    gpu.inject(torch.from_numpy(src64).cuda(), 256, dst, 4)
    assert np.array_equal(dst.cpu().numpy(), src[::4, ::4])


def test_learned_gain_held_out(gpu):
    """The committed, GPU-trained corrector on a held-out seed: the corrected 513^2 run beats the
    plain 513^2 run against the 2049^2 plain run at t = 20 (relative L2 on the 513^2 nodes)."""
    from paper_1109_1027_amd import corrector as K
    params, scale = K.load_weights()
    say("[case] learned corrector gain, held-out seed 9001")
    snaps, _ = K.fine_trajectory(9001, snapshots=False)
    R = snaps[-1].cpu().numpy().astype(np.complex128)
    plain, _, _ = K.plain_run(9001, 512)
    learned, _ = K.learned_run(9001, params, scale)
    e_plain, e_learned = K.rel(plain, R), K.rel(learned, R)
    say(f"[result] E_plain(513^2) {e_plain:.3e}, E_learned {e_learned:.3e}, gain {e_plain / e_learned:.2f}")
    assert e_learned < 0.8 * e_plain
