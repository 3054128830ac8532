"""Pins of the Dirichlet closure (Sec. 3.2, Eqs. dbc_lap, dbc_ut) at NON-ZERO boundary values.

Every configuration and every figure of the paper has Psi_b = 0, where the closure value
D_b = -(s|Psi_b|^2 - V_b) Psi_b / a vanishes whatever the rule.  These tests use stationary
exact solutions of Eq. NLSE whose boundary values are not zero, so the rule itself is
exercised:

* a plane wave Psi = exp(i k.r) with s = 0 and the constant potential V = -a |k|^2:
  a Lap Psi = -a |k|^2 Psi = V Psi, hence Psi_t = 0 and |Psi_b| = 1;
* a real positive product f = prod_a (1.2 + 0.5 sin(k_a x_a + phi_a)) times a constant phase,
  with V = s f^2 + a Lap(f) / f: then a Lap f - V f + s f^3 = 0, Psi_t = 0, and the closure
  involves s, |Psi_b|^2 and V_b together.

For both, Eq. dbc_lap gives the exact Laplacian on every boundary node.  The whole RK4 run
(Eq. RK4) then converges to the stationary field at fourth order in 1D, 2D and 3D, for the
single-storage, per-axis and non-compact forms.  A sign slip or a dropped term in the closure
leaves an O(1) error in the step-2 combination next to the boundary, which stops the
convergence (checked by hand by planting such slips in the oracle).
"""
import numpy as np
import pytest


def _coords(dim, n, x0, h):
    """(x, y, z) node coordinates on the [z][y][x] grid of n intervals per axis."""
    ii = np.indices((n + 1,) * dim).astype(float) * h + x0
    return ii[::-1]


def plane_wave(orc, dim, n, lap="2shoc", L=3.0, a=0.7):
    h = L / n
    X = _coords(dim, n, -0.3, h)
    k = [1.3, -0.8, 0.6][:dim]
    psi = np.exp(1j * sum(k[i] * X[i] for i in range(dim)))
    V = np.full(psi.shape, -a * sum(q * q for q in k))
    exact_lap = -sum(q * q for q in k) * psi
    return orc.Problem(dim, n, h, a, 0.0, V, lap=lap), psi, exact_lap


def real_product(orc, dim, n, lap="2shoc", L=3.0, a=0.6, s=0.5):
    h = L / n
    X = _coords(dim, n, -0.4, h)
    k, ph = [1.1, 0.9, 1.3][:dim], [0.3, 1.0, -0.5][:dim]
    fa = [1.2 + 0.5 * np.sin(k[i] * X[i] + ph[i]) for i in range(dim)]
    fa2 = [-0.5 * k[i] ** 2 * np.sin(k[i] * X[i] + ph[i]) for i in range(dim)]   # f_a''
    f = np.prod(fa, axis=0)
    lapf = sum(fa2[i] * f / fa[i] for i in range(dim))
    V = s * f * f + a * lapf / f
    phase = np.exp(0.4j)
    return orc.Problem(dim, n, h, a, s, V, lap=lap), f * phase, lapf * phase


CASES = {"plane_wave": plane_wave, "real_product": real_product}


def _boundary_mask(shape):
    m = np.zeros(shape, dtype=bool)
    for ax in range(len(shape)):
        idx = [slice(None)] * len(shape)
        idx[ax] = 0
        m[tuple(idx)] = True
        idx[ax] = -1
        m[tuple(idx)] = True
    return m


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("dim,n", [(1, 20), (2, 12), (3, 8)])
def test_boundary_value_is_exact_laplacian(orc, case, dim, n):
    """Eq. dbc_lap on a stationary solution: D_b equals the exact Laplacian on every boundary
    node, and F_b = 0 (Eq. dbc_ut)."""
    P, psi, exact_lap = CASES[case](orc, dim, n)
    D = P.step1(psi)
    m = _boundary_mask(psi.shape)
    assert np.abs(psi[m]).min() > 0.1          # the boundary values really are non-zero
    np.testing.assert_allclose(D[m], exact_lap[m], rtol=0, atol=1e-13 * np.abs(exact_lap).max())
    F = P.rhs(psi)
    assert np.all(F[m] == 0)


def _run_errors(orc, case, dim, ns, lap, t_end=0.5):
    errs = []
    for n in ns:
        P, psi, _ = CASES[case](orc, dim, n, lap=lap)
        nsteps, dt = orc.steps_for(t_end, P.max_dt(psi), 0.5)
        errs.append(orc.rel_l2(P.rk4(psi, nsteps, dt), psi))
    return errs


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("lap", ["2shoc", "axis", "noncompact"])
@pytest.mark.parametrize("dim,ns,min_order", [(1, (16, 32, 64), 3.9), (2, (12, 24, 48), 3.85),
                                              (3, (8, 16), 3.6)])
def test_fourth_order_with_nonzero_dirichlet(orc, case, lap, dim, ns, min_order):
    """The RK4 run keeps the stationary field to fourth order in h (the error falls ~16x per
    halving) although every boundary node is non-zero."""
    errs = _run_errors(orc, case, dim, ns, lap)
    orders = [np.log(errs[i] / errs[i + 1]) / np.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]
    assert orders[-1] >= min_order, (errs, orders)
    assert errs[-1] < 1e-3


@pytest.mark.parametrize("dim,n", [(1, 24), (2, 14), (3, 8)])
def test_forms_agree_on_nonzero_dirichlet_run(orc, dim, n):
    """Whole runs of the three fourth-order forms agree to round-off for the non-zero boundary
    case (the per-axis closure and the non-compact ghost both reduce to Eq. dbc_lap)."""
    outs = []
    for lap in ("2shoc", "axis", "noncompact"):
        P, psi, _ = real_product(orc, dim, n, lap=lap)
        nsteps, dt = orc.steps_for(0.2, P.max_dt(psi), 0.5)
        outs.append(P.rk4(psi, nsteps, dt))
    for o in outs[1:]:
        assert orc.rel_l2(o, outs[0]) < 1e-13
