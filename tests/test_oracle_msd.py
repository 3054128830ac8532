"""Pins of the oracle's modulus-squared Dirichlet (MSD) rule in 2D and 3D.

The paper gives the MSD rule (Sec. 3.2, Eqs. msdbc_ut, msdbc_lap, nbnb1) with b-1 the nearest
interior node in the normal direction, and notes that it carries over to several dimensions; its
tests use it in 1D only (Sec. 4.1, pinned in test_oracle_paper.py by the Fig. 1 orders).  The
multi-D oracle takes b-1 as the closest interior node (the diagonal one at edges and corners).
These tests pin that extension against things the mathematics fixes:

* a stationary dark soliton plane (density constant in time, so MSD is exact on every face, with
  a steep density gradient at one face) converges at fourth order in 2D and 3D, as in 1D;
* a uniform background follows, at every node, the scalar RK4 recursion of Psi' = i s |Psi|^2 Psi;
* the scheme commutes with the grid's reflections and axis permutations;
* the MSD time derivative keeps every boundary density to RK4's local error;
* the per-axis form with the face closure equals the single-storage form;
* the bound's boundary term |B| = (h^2/a)|F_{b-1}/Psi_{b-1}| takes its closed value.
"""
import math

import numpy as np
import pytest

import nlse_inputs as I


def _dark_run(orc, dim, h, t_end=1.0, width=2.0, nst=None):
    n, psi0 = I.dark_plane(dim, h, width=width)
    P = orc.Problem(dim, n, h, 0.5, -1.0, bc="msd")
    if nst is None:
        nst, _ = orc.steps_for(t_end, P.max_dt(psi0))
    out = P.rk4(psi0, nst, t_end / nst)
    _, exact = I.dark_plane(dim, h, t=t_end, width=width)
    return orc.rel_l2(out, exact), nst


@pytest.mark.parametrize("dim,hs,width", [(2, (0.25, 0.125), 2.0), (3, (0.25, 0.125), 1.0)])
def test_msd_dark_plane_fourth_order(orc, dim, hs, width):
    """Fourth order with MSD on every face, notch 1.5 from the x = lo face.  A sign slip in the
    (N_{b-1} - N_b)/a term of Eq. msdbc_lap drops the order to 3 and raises the error tenfold."""
    (e1, n1), (e2, _) = (_dark_run(orc, dim, h, width=width) for h in hs)
    p = math.log(e1 / e2) / math.log(hs[0] / hs[1])
    assert 3.9 < p < 4.1, (e1, e2, p)
    # and the error stays below that of the 1D run on the same x grid with the same steps (the
    # nodes on the faces normal to y and z keep their density, which only lowers it)
    e1d, _ = _dark_run(orc, 1, hs[0], nst=n1)
    assert e1 < 1.2 * e1d, (e1, e1d)


def _scalar_rk4(z, s, k, nsteps):
    f = lambda u: 1j * s * abs(u) ** 2 * u
    for _ in range(nsteps):
        k1 = f(z)
        k2 = f(z + 0.5 * k * k1)
        k3 = f(z + 0.5 * k * k2)
        k4 = f(z + k * k3)
        z = z + (k / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return z


@pytest.mark.parametrize("dim", [2, 3])
def test_msd_uniform_background_scalar_rk4(orc, dim):
    """Every D vanishes, every boundary D_b and F_b reduce to the interior values: each node
    follows the scalar RK4 of Psi' = i s |Psi|^2 Psi.  A boundary rule that froze the boundary
    (e.g. Re instead of Im in Eq. msdbc_ut) fails here."""
    n = (7, 6, 5)[:dim]
    z0 = 0.8 * np.exp(0.3j)
    psi = np.full(tuple(v + 1 for v in reversed(n)), z0)
    P = orc.Problem(dim, n, 0.5, 0.5, -1.0, bc="msd")
    k = 0.4 * P.max_dt(psi)
    out = P.rk4(psi, 40, k)
    ref = _scalar_rk4(z0, -1.0, k, 40)
    assert np.max(np.abs(out - ref)) < 1e-14
    # the bound's boundary term: |F_{b-1}/Psi_{b-1}| = |s| |z0|^2
    _, aux = P.max_dt(psi, return_aux=True)
    assert aux[2] == pytest.approx(0.25 / 0.5 * 0.64, rel=1e-14)


def _rough(shape, seed):
    rng = np.random.default_rng(seed)
    return 1.0 + 0.2 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def test_msd_symmetries_2d(orc):
    """Reflections along x and y, and the transposition of a square grid, commute with the scheme:
    a mistake on one face only (a wrong b-1 on the far face, an edge rule applied on one side)
    breaks them."""
    P = orc.Problem(2, (9, 7), 0.3, 0.7, -1.3, bc="msd")
    psi = _rough((8, 10), 1)
    out = P.rk4(psi, 6, 0.004)
    for ax in (0, 1):
        f = P.rk4(np.flip(psi, ax), 6, 0.004)
        assert np.max(np.abs(f - np.flip(out, ax))) < 1e-13
    Q = orc.Problem(2, 8, 0.3, 0.7, -1.3, bc="msd")
    sq = _rough((9, 9), 2)
    assert np.max(np.abs(Q.rk4(sq.T, 6, 0.004) - Q.rk4(sq, 6, 0.004).T)) < 1e-13


def test_msd_symmetries_3d(orc):
    P = orc.Problem(3, (6, 5, 4), 0.3, 0.7, -1.3, bc="msd")
    psi = _rough((5, 6, 7), 3)
    out = P.rk4(psi, 4, 0.003)
    for ax in (0, 1, 2):
        f = P.rk4(np.flip(psi, ax), 4, 0.003)
        assert np.max(np.abs(f - np.flip(out, ax))) < 1e-13
    Q = orc.Problem(3, 5, 0.3, 0.7, -1.3, bc="msd")
    cube = _rough((6, 6, 6), 4)
    ref = Q.rk4(cube, 4, 0.003)
    for perm in ((0, 2, 1), (2, 1, 0), (1, 2, 0)):
        got = Q.rk4(np.ascontiguousarray(cube.transpose(perm)), 4, 0.003)
        assert np.max(np.abs(got - ref.transpose(perm))) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_msd_boundary_density_kept(orc, dim):
    """Eq. msdbc_ut makes d|Psi_b|^2/dt vanish; RK4 keeps it to its O(k^5) local error per step,
    far below how much the interior moves."""
    n = (12, 10, 8)[:dim]
    shape = tuple(v + 1 for v in reversed(n))
    h = 0.4
    co = np.meshgrid(*[h * np.arange(m) for m in shape], indexing="ij")
    phase = sum((0.3 + 0.2 * i) * c for i, c in enumerate(co))
    # smooth data: the boundary phase rate changes little between the RK4 stages (on rough data
    # k |F_{b-1}/Psi_{b-1}| is O(1) at the bound and the stages no longer compose to a rotation)
    psi = 1.0 + 0.3 * np.exp(1j * phase) * np.cos(0.5 * co[-1])
    P = orc.Problem(dim, n, h, 0.5, -1.0, bc="msd")
    k = 0.5 * P.max_dt(psi)
    out = P.rk4(psi, 20, k)
    bmask = np.zeros(shape, bool)
    for ax in range(dim):
        sl = [slice(None)] * dim
        sl[ax] = 0
        bmask[tuple(sl)] = True
        sl[ax] = -1
        bmask[tuple(sl)] = True
    dens = np.abs(out) ** 2 - np.abs(psi) ** 2
    assert np.max(np.abs(dens[bmask])) < 2e-6
    assert np.max(np.abs(dens[~bmask])) > 0.1


@pytest.mark.parametrize("dim", [2, 3])
def test_msd_per_axis_equals_single_storage(orc, dim):
    """With the face closure D^a_q = Lap_b(q) - (tangential second differences), the per-axis form
    (Eqs. 2d2shocMs1-2 / 3d2shocMs1-2) equals the single-storage one for any boundary value,
    including the MSD one, to round-off."""
    n = (9, 8, 7)[:dim]
    psi = _rough(tuple(v + 1 for v in reversed(n)), 6)
    P = orc.Problem(dim, n, 0.3, 0.5, -1.0, bc="msd")
    a = P.laplacian(psi)
    b = P.with_lap("axis").laplacian(psi)
    assert np.max(np.abs(a - b)) < 1e-11 * np.max(np.abs(a))


def test_msd_symmetry_with_potential(orc):
    """The same reflection symmetry with a potential even in x: V enters N at b and b-1."""
    n = (9, 7)
    x = 0.3 * np.arange(10) - 1.35
    y = 0.3 * np.arange(8)
    V = 0.4 * x[None, :] ** 2 + 0.2 * y[:, None]
    P = orc.Problem(2, n, 0.3, 0.7, -1.3, V=V, bc="msd")
    psi = _rough((8, 10), 7)
    out = P.rk4(psi, 6, 0.004)
    f = P.rk4(np.flip(psi, 1), 6, 0.004)
    assert np.max(np.abs(f - np.flip(out, 1))) < 1e-13
    # and V matters: the run differs from the one without it
    Q = orc.Problem(2, n, 0.3, 0.7, -1.3, bc="msd")
    assert np.max(np.abs(Q.rk4(psi, 6, 0.004) - out)) > 1e-4
