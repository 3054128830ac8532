"""CPU reference of the learned coarse-grid corrector -- TEST INFRASTRUCTURE ONLY.

The corrector is a 3-layer 3x3 convolutional network on the coarse 2D field:

    A0 = bf16(features(Psi))                       [H, W, 8]
    Z1 = conv3x3(A0, W1) + b1,  A1 = bf16(silu(Z1))  [H, W, 32]
    Z2 = conv3x3(A1, W2) + b2,  A2 = bf16(silu(Z2))  [H, W, 32]
    Y  = conv3x3(A2, W3) + b3                      [H, W, 2]   (FP32, not rounded)
    Psi <- Psi + scale * (Y0 + i Y1) on interior nodes

with zero padding, weights rounded to bf16 (round to nearest even) before use and
sums accumulated exactly (FP64 here; FP32 on the GPU).  Training minimises the
mean squared error between Y and target/scale over interior nodes; the backward
pass treats the bf16 roundings as the identity (straight through) and rounds the
propagated gradients dY, dZ2, dZ1 to bf16 where the GPU does (emulate=True).

This is a plain definition written out with numpy loops over the nine taps; it
shares no code with the GPU library.  Pins (tests/test_oracle_conv.py): the
forward convolution equals scipy.signal.correlate (an independent routine), and
the analytic gradients equal central finite differences of the FP64 loss.
The trained weights themselves are parity unpinned (judged by the gain test).
"""
from __future__ import annotations

import numpy as np

C_IN, HIDDEN, C_OUT = 8, 32, 2
LAP_SCALE, V_SCALE = 16.0, 0.25
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]   # tap t = (dy+1)*3 + (dx+1)


def bf16(x):
    """Round float values to bfloat16 (round to nearest even), returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(psi, V, h, emulate=True):
    """Input channels of the corrector at every node of a 2D field [H, W]:
    Re Psi, Im Psi, 16 Re(h^2 L Psi), 16 Im(h^2 L Psi), |Psi|^2, V/4, 0, 0 with L the
    five-point Laplacian (zero outside the grid), evaluated in FP32 when emulating."""
    dt = np.complex64 if emulate else np.complex128
    p = np.asarray(psi).astype(dt)
    pad = np.zeros((p.shape[0] + 2, p.shape[1] + 2), dtype=dt)
    pad[1:-1, 1:-1] = p
    lap5 = pad[:-2, 1:-1] + pad[2:, 1:-1] + pad[1:-1, :-2] + pad[1:-1, 2:] - 4 * p   # h^2 * Laplacian
    f = np.zeros(p.shape + (C_IN,), dtype=np.float64)
    f[..., 0] = p.real
    f[..., 1] = p.imag
    f[..., 2] = LAP_SCALE * lap5.real
    f[..., 3] = LAP_SCALE * lap5.imag
    f[..., 4] = (p.real.astype(np.float64) ** 2 + p.imag.astype(np.float64) ** 2)
    f[..., 5] = V_SCALE * np.asarray(V, dtype=np.float64)
    if emulate:
        f = f.astype(np.float32).astype(np.float64)
    return f


def conv3x3(X, W, b):
    """Z[y, x, n] = b[n] + sum_t sum_c X[y+dy_t, x+dx_t, c] W[n, t, c] (zero padding)."""
    H, Wd, _ = X.shape
    Xp = np.zeros((H + 2, Wd + 2, X.shape[2]))
    Xp[1:-1, 1:-1] = X
    Z = np.broadcast_to(np.asarray(b, dtype=np.float64), (H, Wd, W.shape[0])).copy()
    for t, (dy, dx) in enumerate(TAPS):
        Z += Xp[1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd] @ W[:, t, :].T
    return Z


def conv3x3_transpose(G, W):
    """Adjoint of conv3x3 in its input: dX[q, c] = sum_t sum_n G[q - off_t, n] W[n, t, c]."""
    H, Wd, _ = G.shape
    Gp = np.zeros((H + 2, Wd + 2, G.shape[2]))
    Gp[1:-1, 1:-1] = G
    dX = np.zeros((H, Wd, W.shape[2]))
    for t, (dy, dx) in enumerate(TAPS):
        dX += Gp[1 - dy:1 - dy + H, 1 - dx:1 - dx + Wd] @ W[:, t, :]
    return dX


def weight_grad(X, G):
    """dW[n, t, c] = sum_p G[p, n] X[p + off_t, c]."""
    H, Wd, C = X.shape
    Xp = np.zeros((H + 2, Wd + 2, C))
    Xp[1:-1, 1:-1] = X
    out = np.zeros((G.shape[2], 9, C))
    for t, (dy, dx) in enumerate(TAPS):
        out[:, t, :] = G.reshape(-1, G.shape[2]).T @ Xp[1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd].reshape(-1, C)
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def interior_mask(H, W):
    m = np.zeros((H, W), dtype=bool)
    m[1:-1, 1:-1] = True
    return m


def init_params(seed=0):
    """Seeded initial FP32 master weights (He-style scale; last layer small)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.standard_normal((HIDDEN, 9, C_IN)) * np.sqrt(2.0 / (9 * C_IN)),
         "b1": np.zeros(HIDDEN),
         "W2": rng.standard_normal((HIDDEN, 9, HIDDEN)) * np.sqrt(2.0 / (9 * HIDDEN)),
         "b2": np.zeros(HIDDEN),
         "W3": rng.standard_normal((C_OUT, 9, HIDDEN)) * 1e-3,
         "b3": np.zeros(C_OUT)}
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def forward(params, X0, emulate=True):
    """Returns Y and the cached activations.  X0: features [H, W, 8]."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    A0 = r(X0)
    Z1 = conv3x3(A0, r(params["W1"]), params["b1"])
    A1 = r(silu(Z1))
    Z2 = conv3x3(A1, r(params["W2"]), params["b2"])
    A2 = r(silu(Z2))
    Y = conv3x3(A2, r(params["W3"]), params["b3"])
    return Y, {"A0": A0, "Z1": Z1, "A1": A1, "Z2": Z2, "A2": A2}


def loss_and_grads(params, X0, T, emulate=True):
    """MSE over interior nodes and both output channels, and its gradients (FP64)."""
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    Y, c = forward(params, X0, emulate)
    H, Wd = Y.shape[:2]
    m = interior_mask(H, Wd)[..., None]
    count = m.sum() * C_OUT
    d = (Y - T) * m
    loss = float(np.sum(d * d) / count)
    dY = r(2.0 * d / count)
    g = {"W3": weight_grad(c["A2"], dY), "b3": dY.sum(axis=(0, 1))}
    dZ2 = r(conv3x3_transpose(dY, r(params["W3"])) * dsilu(c["Z2"]))
    g["W2"] = weight_grad(c["A1"], dZ2)
    g["b2"] = dZ2.sum(axis=(0, 1))
    dZ1 = r(conv3x3_transpose(dZ2, r(params["W2"])) * dsilu(c["Z1"]))
    g["W1"] = weight_grad(c["A0"], dZ1)
    g["b1"] = dZ1.sum(axis=(0, 1))
    return loss, g, Y
