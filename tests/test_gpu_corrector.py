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


# ----------------------------------------------------------------------------------------
# Layer-by-layer parity.  Each GPU stage runs on seeded host tensors (nlse_corr_tensor /
# nlse_corr_stage) and is compared with oracle/conv.py on the same tensors.  FP32 sums of
# K products (the MFMA accumulation, and the weight gradients' fixed-order reduction) are
# within gamma_K * sum|terms| of the exact FP64 value, gamma_K = K u / (1 - K u), u = 2^-24
# (the standard bound for any summation order); a bf16 output is within half a bf16 unit
# (2^-8 relative) of the exact value, widened by the error of the FP32 quantity it rounds
# and 16 u for the hardware exponential and reciprocal in silu.

U32 = 2.0 ** -24


def gamma(k):
    return k * U32 / (1.0 - k * U32)


def to_bits(x):
    """float64 values -> raw bf16 patterns (round to nearest even, as conv.bf16)."""
    f = conv.bf16(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def from_bits(u):
    return (np.asarray(u, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def rand_bf16(rng, shape, scale=1.0):
    return to_bits(rng.standard_normal(shape) * scale)


def check_fp32_sum(got, exact, abs_terms, k, what):
    err = np.abs(got.astype(np.float64) - exact)
    bound = gamma(k) * abs_terms + U32 * np.abs(exact)
    worst = float(np.max(err / np.maximum(bound, 1e-300)))
    scale = float(np.max(np.abs(exact)))
    say(f"[result] {what}: max |err| {err.max():.3e} (max |value| {scale:.3e}), worst err/bound {worst:.3f}")
    assert np.all(err <= bound), what


def check_bf16(got_bits, exact, slack, what):
    got = from_bits(got_bits)
    err = np.abs(got - exact)
    bound = 2.0 ** -8 * (np.abs(exact) + slack) + slack
    worst = float(np.max(err / np.maximum(bound, 1e-300)))
    say(f"[result] {what}: max |err| {err.max():.3e}, worst err/bound {worst:.3f}")
    assert np.all(err <= bound), what


B_L, H_L, W_L = 2, 21, 45   # ragged: W is not a multiple of the 32-pixel wave tile


def layer_setup(gpu, seed):
    p = nontrivial_params(seed)
    m = gpu.Corrector(H_L, W_L, max_batch=B_L)
    m.set_params(flat(p), 1.0)
    return m, p


@pytest.mark.parametrize("layer", [1, 2, 3])
def test_layer_forward_fp32_accumulators(gpu, layer):
    """Z1 / Z2 / Y from seeded bf16 inputs: FP32 MFMA sums within gamma_K sum|terms| of the FP64
    convolution; A1 / A2 within half a bf16 unit of bf16(silu(Z))."""
    rng = np.random.default_rng(100 + layer)
    m, p = layer_setup(gpu, 40 + layer)
    cin = 8 if layer == 1 else 32
    x = rand_bf16(rng, (B_L, H_L, W_L, cin))
    if layer == 1:
        x[..., 6:] = 0   # the two unused feature channels
    m.put_tensor({1: "X0", 2: "A1", 3: "A2"}[layer], x)
    m.stage(f"fwd{layer}", B_L)
    W = conv.bf16(p[f"W{layer}"])
    b = p[f"b{layer}"]
    cout = W.shape[0]
    xf = from_bits(x)
    k = 9 * cin + 1
    if layer < 3:
        Z = m.get_tensor(f"Z{layer}", (B_L, H_L, W_L, cout), np.float32)
        A = m.get_tensor(f"A{layer}", (B_L, H_L, W_L, cout), np.uint16)
    else:
        Z = m.get_tensor("Y", (B_L, H_L, W_L, cout), np.float32)
    for i in range(B_L):
        ex = conv.conv3x3(xf[i], W, b)
        terms = conv.conv3x3(np.abs(xf[i]), np.abs(W), np.abs(b))
        check_fp32_sum(Z[i], ex, terms, k, f"layer {layer} FP32 sums, sample {i}")
        if layer < 3:
            zerr = gamma(k) * terms + U32 * np.abs(ex)
            # silu' is bounded by 1.1: the FP32 error of Z moves silu by at most 1.1 zerr
            check_bf16(A[i], conv.silu(ex), 1.1 * zerr + 16 * U32 * np.abs(conv.silu(ex)),
                       f"layer {layer} bf16 activations, sample {i}")


@pytest.mark.parametrize("layer", [3, 2, 1])
def test_layer_weight_gradients(gpu, layer):
    """dW, db of each layer from seeded bf16 inputs and output gradients: the FP32 reduction
    over the batch's pixels within gamma_K sum|terms| of the FP64 sums."""
    rng = np.random.default_rng(200 + layer)
    m, p = layer_setup(gpu, 50 + layer)
    cin = 8 if layer == 1 else 32
    x = rand_bf16(rng, (B_L, H_L, W_L, cin))
    if layer == 1:
        x[..., 6:] = 0
    if layer == 3:
        g = np.zeros((B_L, H_L, W_L, 8), np.uint16)
        g[..., :2] = rand_bf16(rng, (B_L, H_L, W_L, 2), 1e-2)
        cout = 2
    else:
        g = rand_bf16(rng, (B_L, H_L, W_L, 32), 1e-2)
        cout = 32
    m.put_tensor({1: "X0", 2: "A1", 3: "A2"}[layer], x)
    m.put_tensor({1: "dZ1", 2: "dZ2", 3: "dY"}[layer], g)
    m.put_tensor("grads", np.zeros(m.nparam, np.float32))
    m.stage(f"wgrad{layer}", B_L)
    gr = m.get_tensor("grads", (m.nparam,), np.float32).astype(np.float64)
    xf, gf = from_bits(x), from_bits(g)[..., :cout]
    ex_w = sum(conv.weight_grad(xf[i], gf[i]) for i in range(B_L))
    ab_w = sum(conv.weight_grad(np.abs(xf[i]), np.abs(gf[i])) for i in range(B_L))
    ex_b = gf.sum(axis=(0, 1, 2))
    ab_b = np.abs(gf).sum(axis=(0, 1, 2))
    offs = {"W1": (0, 2304), "b1": (2304, 2336), "W2": (2336, 11552), "b2": (11552, 11584),
            "W3": (11584, 12160), "b3": (12160, 12162)}
    k = B_L * H_L * W_L
    a, e = offs[f"W{layer}"]
    check_fp32_sum(gr[a:e], ex_w.ravel(), ab_w.ravel(), k, f"dW{layer}")
    a, e = offs[f"b{layer}"]
    check_fp32_sum(gr[a:e], ex_b, ab_b, k, f"db{layer}")


@pytest.mark.parametrize("layer", [3, 2])
def test_layer_input_gradients(gpu, layer):
    """dZ2 = bf16(conv^T(dY, W3) silu'(Z2)) and dZ1 = bf16(conv^T(dZ2, W2) silu'(Z1)) from seeded
    inputs: within half a bf16 unit of the exact value, widened by the FP32 sum's bound."""
    rng = np.random.default_rng(300 + layer)
    m, p = layer_setup(gpu, 60 + layer)
    if layer == 3:
        g = np.zeros((B_L, H_L, W_L, 8), np.uint16)
        g[..., :2] = rand_bf16(rng, (B_L, H_L, W_L, 2), 1e-2)
        gf = from_bits(g)[..., :2]
        k = 9 * 8
    else:
        g = rand_bf16(rng, (B_L, H_L, W_L, 32), 1e-2)
        gf = from_bits(g)
        k = 9 * 32
    z = (rng.standard_normal((B_L, H_L, W_L, 32)) * 2.0).astype(np.float32)
    m.put_tensor({3: "dY", 2: "dZ2"}[layer], g)
    m.put_tensor({3: "Z2", 2: "Z1"}[layer], z)
    m.stage(f"bwd{layer}", B_L)
    out = m.get_tensor({3: "dZ2", 2: "dZ1"}[layer], (B_L, H_L, W_L, 32), np.uint16)
    W = conv.bf16(p[f"W{layer}"])
    for i in range(B_L):
        s = conv.conv3x3_transpose(gf[i], W)
        s_abs = conv.conv3x3_transpose(np.abs(gf[i]), np.abs(W))
        d = conv.dsilu(z[i].astype(np.float64))
        ex = s * d
        slack = (gamma(k) * s_abs + U32 * np.abs(s)) * np.abs(d) + 16 * U32 * np.abs(ex)
        check_bf16(out[i], ex, slack, f"input gradient of layer {layer}, sample {i}")
