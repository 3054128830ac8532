"""Pins of the oracle's Laplacian against facts fixed by the paper and by calculus.

* Polynomial exactness (Sec. 2.1: the double difference is fourth-order; the combined
  stencil is the five-point fourth-order stencil, whose leading error is -(h^4/90) f^(6)).
* Equivalences the paper states: 2SHOC == non-compact stencil (Sec. 2.1, Eq. 2dnonhoc,
  Sec. 2.3) and single-storage == per-axis (Sec. 2.2-2.3).
* The operator in closed form under Dirichlet 0: per axis T - (h^2/12) T^2 with
  T = tridiag(1, -2, 1)/h^2 (Kronecker sums in 2D/3D), built here without the oracle.
* The boundary rules (Sec. 3.2, Eqs. dbc_lap, msdbc_lap).
"""
import math

import numpy as np
import pytest

rng = np.random.default_rng(1234)


def rand_field(shape, zero_boundary=True):
    f = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    if zero_boundary:
        m = np.zeros(shape, dtype=bool)
        for ax in range(len(shape)):
            idx = [slice(None)] * len(shape)
            idx[ax] = 0
            m[tuple(idx)] = True
            idx[ax] = -1
            m[tuple(idx)] = True
        f[m] = 0
    return f


def inner(a, dim, w=2):
    return a[(slice(w, -w),) * dim]


# ----------------------------------------------------------------- 1D --

@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_1d_polynomial_exact(orc, p):
    n, h = 40, 0.1
    x = -2.0 + h * np.arange(n + 1)
    f = (x ** p).astype(np.complex128) * (1 + 0.5j)
    exact = (p * (p - 1) * x ** (p - 2) if p >= 2 else 0 * x) * (1 + 0.5j)
    P = orc.Problem(1, n, h, 1.0, 0.0)
    lap = P.laplacian(f)
    # nodes >= 2 from the ends never read a boundary closure value
    np.testing.assert_allclose(lap[2:-2], exact[2:-2], rtol=0, atol=1e-9 * max(1, np.abs(exact).max()))


def test_1d_degree6_error_term(orc):
    """For x^6 the five-point fourth-order stencil errs by exactly -(h^4/90)*720."""
    n, h = 40, 0.1
    x = -2.0 + h * np.arange(n + 1)
    lap = orc.Problem(1, n, h, 1.0, 0.0).laplacian(x ** 6 + 0j)
    err = lap.real - 30 * x ** 4
    np.testing.assert_allclose(err[2:-2], -(h ** 4 / 90.0) * 720.0, rtol=1e-7)


def test_1d_equals_five_point_stencil(orc):
    n, h = 30, 0.37
    f = rand_field((n + 1,))
    lap = orc.Problem(1, n, h, 1.0, 0.0).laplacian(f)
    five = (-f[4:] + 16 * f[3:-1] - 30 * f[2:-2] + 16 * f[1:-3] - f[:-4]) / (12 * h * h)
    np.testing.assert_allclose(lap[2:-2], five, rtol=1e-12, atol=1e-12 * np.abs(five).max())


def _tmat(m, h):
    """Second-difference matrix on m interior nodes with zero Dirichlet values."""
    return (np.diag(-2.0 * np.ones(m)) + np.diag(np.ones(m - 1), 1) + np.diag(np.ones(m - 1), -1)) / h ** 2


def _closed_form_operator(dim, n, h):
    m = n - 1
    T = _tmat(m, h)
    A1 = T - (h * h / 12.0) * T @ T
    I = np.eye(m)
    if dim == 1:
        return A1
    if dim == 2:
        return np.kron(I, A1) + np.kron(A1, I)          # x fastest: x-part acts on the last index
    return np.kron(np.kron(I, I), A1) + np.kron(np.kron(I, A1), I) + np.kron(np.kron(A1, I), I)


def _oracle_operator(orc, dim, n, h, lap="2shoc"):
    P = orc.Problem(dim, n, h, 1.0, 0.0, lap=lap)
    shape = (n + 1,) * dim
    inner_idx = np.argwhere(np.ones((n - 1,) * dim, dtype=bool)) + 1
    M = np.zeros((len(inner_idx), len(inner_idx)))
    for c, idx in enumerate(inner_idx):
        e = np.zeros(shape, dtype=np.complex128)
        e[tuple(idx)] = 1.0
        out = P.laplacian(e)
        M[:, c] = out[(slice(1, -1),) * dim].real.ravel()
    return M


@pytest.mark.parametrize("dim,n", [(1, 9), (2, 7), (3, 5)])
@pytest.mark.parametrize("lap", ["2shoc", "axis", "noncompact"])
def test_operator_closed_form_dirichlet0(orc, dim, n, lap):
    """Under Dirichlet 0 the 2SHOC operator is the Kronecker sum of T - (h^2/12) T^2 per axis."""
    h = 0.3
    M = _oracle_operator(orc, dim, n, h, lap)
    ref = _closed_form_operator(dim, n, h)
    np.testing.assert_allclose(M, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    np.testing.assert_allclose(M, M.T, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("dim,n", [(1, 64), (2, 24), (3, 10)])
def test_spectrum_bounded_by_gmax(orc, dim, n):
    """h^2 * spectrum lies in [-G_max, 0) with G_max = 64/12, 128/12, 192/12 (Table t:sumresults)."""
    h = 1.0
    M = _oracle_operator(orc, dim, n, h) if dim < 3 else _closed_form_operator(dim, n, h)
    ev = np.linalg.eigvalsh(0.5 * (M + M.T)) * h * h
    gmax = 64.0 * dim / 12.0
    assert ev.max() < 0
    assert ev.min() > -gmax
    assert ev.min() < -0.95 * gmax


# ---------------------------------------------------------- 2D and 3D --

@pytest.mark.parametrize("dim", [2, 3])
def test_multid_polynomial_exact(orc, dim):
    n, h = 12 if dim == 3 else 20, 0.125
    g = [(-0.7 + h * np.arange(n + 1))] * dim
    mesh = np.meshgrid(*g, indexing="ij")[::-1]   # (x, y[, z]) in [z][y][x]
    x, y = mesh[0], mesh[1]
    z = mesh[2] if dim == 3 else 0 * x
    f = x ** 5 + 2 * y ** 4 * x ** 3 - 3 * z ** 5 * y ** 2 + x * y * z + 1.5j * (y ** 5 - x ** 2 * z ** 3)
    lap_exact = (20 * x ** 3 + 24 * y ** 2 * x ** 3 + 12 * y ** 4 * x - 60 * z ** 3 * y ** 2 - 6 * z ** 5
                 + 1.5j * (20 * y ** 3 - 2 * z ** 3 - 6 * x ** 2 * z))
    for lap in ("2shoc", "axis", "noncompact"):
        out = orc.Problem(dim, n, h, 1.0, 0.0, lap=lap).laplacian(f)
        np.testing.assert_allclose(inner(out, dim), inner(lap_exact, dim), rtol=0,
                                   atol=1e-9 * np.abs(lap_exact).max(), err_msg=lap)


@pytest.mark.parametrize("dim,n", [(2, 17), (3, 9)])
def test_single_storage_equals_per_axis_any_boundary(orc, dim, n):
    """Single-storage and per-axis 2SHOC agree to round-off for arbitrary boundary values
    and a non-zero nonlinearity and potential (the boundary closure enters both)."""
    h = 0.21
    f = rand_field((n + 1,) * dim, zero_boundary=False)
    V = rng.uniform(0, 2, (n + 1,) * dim)
    a = orc.Problem(dim, n, h, 0.7, -1.3, V, lap="2shoc").laplacian(f)
    b = orc.Problem(dim, n, h, 0.7, -1.3, V, lap="axis").laplacian(f)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("dim,n", [(1, 33), (2, 17), (3, 9)])
def test_2shoc_equals_noncompact_odd_ghosts(orc, dim, n):
    """With zero boundary values the compact scheme equals the non-compact stencil with odd ghosts."""
    h = 0.4
    f = rand_field((n + 1,) * dim)
    a = orc.Problem(dim, n, h, 1.0, 2.0, lap="2shoc").laplacian(f)
    b = orc.Problem(dim, n, h, 1.0, 2.0, lap="noncompact").laplacian(f)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("dim,n", [(1, 33), (2, 17), (3, 9)])
def test_2shoc_equals_noncompact_any_dirichlet(orc, dim, n):
    """Sec. 2.1: the two-step scheme is the five-point fourth-order stencil.  Next to a boundary
    node b the five-point stencil reads one node beyond b; the ghost 2 Psi_b - Psi_{b+-1} +
    h^2 D^a_b has the step-1 boundary value D^a_b (Eq. dbc_lap) as its second difference at b,
    so the two agree to round-off for arbitrary Dirichlet values, s and V as well."""
    h = 0.4
    f = rand_field((n + 1,) * dim, zero_boundary=False)
    V = rng.uniform(-1, 2, (n + 1,) * dim)
    a = orc.Problem(dim, n, h, 0.6, -1.7, V, lap="2shoc").laplacian(f)
    b = orc.Problem(dim, n, h, 0.6, -1.7, V, lap="noncompact").laplacian(f)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())


def test_cd_is_second_difference(orc):
    n, h = 12, 0.5
    f = rand_field((n + 1, n + 1))
    out = orc.Problem(2, n, h, 1.0, 0.0, lap="cd").laplacian(f)
    ref = (f[1:-1, 2:] + f[1:-1, :-2] + f[2:, 1:-1] + f[:-2, 1:-1] - 4 * f[1:-1, 1:-1]) / h ** 2
    np.testing.assert_allclose(out[1:-1, 1:-1], ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim,n", [(1, 12), (2, 9), (3, 7)])
def test_cd_quartic_closed_form(orc, dim, n):
    """The second difference of x^4 is 12 x^2 + 2 h^2 exactly, so CD(sum_a x_a^4) =
    12 |r|^2 + 2 d h^2 at every interior node (catches a dropped axis or a wrong scale)."""
    h = 0.25
    idx = np.indices((n + 1,) * dim).astype(float) * h - 0.6   # [z][y][x] order, any origin
    f = np.sum(idx ** 4, axis=0) * (1.0 - 0.5j)
    out = orc.Problem(dim, n, h, 1.0, 0.0, lap="cd").laplacian(f)
    ref = (12.0 * np.sum(idx ** 2, axis=0) + 2.0 * dim * h * h) * (1.0 - 0.5j)
    np.testing.assert_allclose(inner(out, dim, 1), inner(ref, dim, 1), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim,n", [(1, 9), (2, 8), (3, 6)])
def test_noncompact_ghost_closed_form(orc, dim, n):
    """Ghosts with non-zero boundary values, in closed form.  For f = c (sum_a (x_a^2 + c_a x_a)
    + c0) with s = V = 0, Eq. dbc_lap gives Lap_b = 0 on every boundary node, so on a face node
    normal to axis a the per-axis value is D^a_b = 0 - (second differences along the face) =
    -2 c (d - 1) (each tangential x_b^2 differences to 2 c exactly).  The ghost's second
    difference at b is that value, so along an axis on which the node is next to a face the
    five-point difference is (7/6) 2c - (1/12)(2c + D^a_b) = 2c (12 + d)/12 (linear terms and
    constants difference to zero), and 2c deep inside.  Hence
    Lap = c [2 d + (2 d / 12) (number of axes on which the node is next to a face)]."""
    h = 0.3
    ii = np.indices((n + 1,) * dim)
    xs = ii.astype(float) * h
    cf = np.array([0.7, -1.1, 0.4][:dim])
    c = 0.8 + 0.3j
    f = (np.sum(xs ** 2, axis=0) + np.tensordot(cf, xs, axes=1) + 2.5) * c
    out = orc.Problem(dim, n, h, 1.0, 0.0, lap="noncompact").laplacian(f)
    near = np.sum((ii == 1) | (ii == n - 1), axis=0)
    ref = (2.0 * dim + (2.0 * dim / 12.0) * near) * c
    np.testing.assert_allclose(inner(out, dim, 1), inner(ref, dim, 1), rtol=1e-11, atol=1e-11)


def test_3d_edge_neighbours_decoding(orc):
    """The single-storage 3D step 2 touches exactly the 6 face and 12 edge neighbours:
    its response to a delta equals the 13-point non-compact stencil (no corner terms)."""
    n, h = 8, 1.0
    e = np.zeros((n + 1,) * 3, dtype=np.complex128)
    e[4, 4, 4] = 1.0
    out = orc.Problem(3, n, h, 1.0, 0.0).laplacian(e)
    ref = orc.Problem(3, n, h, 1.0, 0.0, lap="noncompact").laplacian(e)
    np.testing.assert_allclose(out, ref, atol=1e-14)
    assert out[4, 4, 4].real == pytest.approx(-3 * 30 / 12)
    assert abs(out[5, 5, 5]) < 1e-15 and abs(out[5, 5, 4]) < 1e-15


# -------------------------------------------------------- boundary rules --

def test_dirichlet_step1_boundary_rule(orc):
    """Eq. dbc_lap: D_b = -(s|Psi_b|^2 - V_b) Psi_b / a; F_b = 0 (Eq. dbc_ut)."""
    n, h, a, s = 10, 0.3, 0.8, 1.7
    f = rand_field((n + 1, n + 1), zero_boundary=False)
    V = rng.uniform(0, 1, f.shape)
    P = orc.Problem(2, n, h, a, s, V)
    D = P.step1(f)
    b = (0, 3)
    assert D[b] == pytest.approx(-(s * abs(f[b]) ** 2 - V[b]) * f[b] / a, rel=1e-14)
    F = P.rhs(f)
    assert np.all(F[0, :] == 0) and np.all(F[:, -1] == 0)


def test_msd_boundary_rules(orc):
    """Eq. msdbc_lap and Eq. msdbc_ut on the 1D dark soliton: the boundary time derivative keeps
    |Psi_b|^2 fixed (Re(conj(Psi_b) F_b) = 0) and F_b / Psi_b is purely imaginary."""
    import nlse_inputs as I
    sp = I.paper_fig1(0.25)
    P = orc.Problem.from_spec(sp)
    F = P.rhs(sp.psi0)
    for b in (0, -1):
        assert abs((np.conj(sp.psi0[b]) * F[b]).real) < 1e-14
    # for the exact travelling solution the boundary phase rate matches the analytic one:
    # Psi_t / Psi at the boundary = i (Omega - c^2/(4a)) + (tanh-term) ~ i(Omega - c^2/4a) far out
    (x,) = sp.grid.coords()
    rate = (F[0] / sp.psi0[0]).imag
    assert rate == pytest.approx(-1.0 - 0.25 / 4.0 + 0.0, abs=2e-3)
    D = P.step1(sp.psi0)
    # Lap Psi_b = [Re(D_1/Psi_1) + (N_1 - N_0)/a] Psi_0
    N = lambda i: sp.s * abs(sp.psi0[i]) ** 2
    exp0 = ((D[1] / sp.psi0[1]).real + (N(1) - N(0)) / sp.a) * sp.psi0[0]
    assert D[0] == pytest.approx(exp0, rel=1e-13)
    # the exact Laplacian of the plane-wave far field is -(c/2a)^2 Psi; the rule reproduces it
    assert D[0] == pytest.approx(-(0.25 ** 2) * sp.psi0[0], rel=2e-3)
