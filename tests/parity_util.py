"""Error measures shared by the GPU parity tests."""
import numpy as np


def rel(a, b):
    """Relative L2 error over all nodes."""
    return float(np.linalg.norm((np.asarray(a, np.complex128) - b).ravel()) / np.linalg.norm(b.ravel()))


def line_err(a, b):
    """Largest relative L2 error over the grid lines along every axis (rows and columns in 2D,
    the three line families in 3D).  A line's error is taken relative to its own norm, or to an
    average line's norm where its own is smaller (boundary lines that hold zeros).  A single wrong
    row or column, which moves the global norm by only about 1/sqrt(lines) of its own error, fails
    this measure at the global tolerance."""
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    d2 = np.abs(a - b) ** 2
    r2 = np.abs(b) ** 2
    worst = 0.0
    for ax in range(b.ndim):
        num = np.sqrt(d2.sum(axis=ax))
        den = np.sqrt(r2.sum(axis=ax))
        floor = np.sqrt(r2.sum()) / np.sqrt(num.size)
        worst = max(worst, float(np.max(num / np.maximum(den, floor))))
    return worst
