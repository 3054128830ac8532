"""Pins of the corrector's CPU reference (oracle/conv.py) against independent routines and calculus:
scipy's 2D correlation, the adjoint identity, finite differences of the loss, torch's bfloat16 cast."""
import numpy as np
import pytest
import scipy.signal

from oracle import conv

rng = np.random.default_rng(3)


def test_conv3x3_equals_scipy_correlate():
    X = rng.standard_normal((7, 9, 5))
    W = rng.standard_normal((4, 9, 5))
    b = rng.standard_normal(4)
    Z = conv.conv3x3(X, W, b)
    for n in range(4):
        ref = b[n] + sum(scipy.signal.correlate2d(X[..., c], W[n, :, c].reshape(3, 3), mode="same")
                         for c in range(5))
        np.testing.assert_allclose(Z[..., n], ref, rtol=1e-12, atol=1e-12)


def test_transpose_is_adjoint():
    X = rng.standard_normal((6, 8, 3))
    G = rng.standard_normal((6, 8, 4))
    W = rng.standard_normal((4, 9, 3))
    lhs = np.sum(conv.conv3x3(X, W, np.zeros(4)) * G)
    rhs = np.sum(X * conv.conv3x3_transpose(G, W))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_weight_grad_is_derivative():
    X = rng.standard_normal((6, 8, 3))
    G = rng.standard_normal((6, 8, 4))
    dW = rng.standard_normal((4, 9, 3))
    lhs = np.sum(conv.weight_grad(X, G) * dW)
    rhs = np.sum(conv.conv3x3(X, dW, np.zeros(4)) * G)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_loss_gradient_finite_differences():
    H, W = 6, 7
    X0 = rng.standard_normal((H, W, conv.C_IN))
    T = rng.standard_normal((H, W, conv.C_OUT))
    p = conv.init_params(seed=5)
    p["W3"] = rng.standard_normal(p["W3"].shape) * 0.3
    p["b1"] = rng.standard_normal(p["b1"].shape) * 0.1
    loss, g, _ = conv.loss_and_grads(p, X0, T, emulate=False)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p[name].shape)
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += eps
            lp = conv.loss_and_grads(q, X0, T, emulate=False)[0]
            q[name][idx] -= 2 * eps
            lm = conv.loss_and_grads(q, X0, T, emulate=False)[0]
            fd = (lp - lm) / (2 * eps)
            assert g[name][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, idx)


def test_bf16_rounding_matches_torch():
    import torch
    x = np.concatenate([rng.standard_normal(10000) * 10 ** rng.uniform(-5, 5, 10000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(conv.bf16(x), ref)


def test_features_channels():
    psi = rng.standard_normal((5, 6)) + 1j * rng.standard_normal((5, 6))
    V = rng.uniform(0, 4, (5, 6))
    f = conv.features(psi, V, 0.1, emulate=False)
    assert f.shape == (5, 6, 8)
    np.testing.assert_allclose(f[..., 4], np.abs(psi) ** 2)
    np.testing.assert_allclose(f[2, 3, 2] / 16, (psi[1, 3] + psi[3, 3] + psi[2, 2] + psi[2, 4] - 4 * psi[2, 3]).real)
    assert np.all(f[..., 6:] == 0)
