"""Pins of the oracle's time stepping, step-size bound and diagnostics.

* One RK4 step of a linear problem equals the degree-4 Taylor polynomial of exp(kA)
  applied to Psi (the stability polynomial of classic RK4, Sec. 3.1), with A built
  here as a dense matrix from the closed-form operator -- not from the oracle.
* A single discrete eigenmode is multiplied by R(iy) = 1 + iy - y^2/2 - i y^3/6 + y^4/24.
* The linear bound Eq. kd2shoclin equals Eq. kdfull at s = V = 0; runs just above / below
  the bound grow / do not grow (Sec. 3.3).
* The paper's own step sizes lie just under the bound (Sec. 4.1-4.3).
* Mass: semi-discrete conservation (symmetric operator) and the RK4 damping |R(iy)|^2.
* Energy: the discrete Hamiltonian of the harmonic-oscillator ground state tends to d * mass.
"""
import json
import math
import os

import numpy as np
import pytest

import nlse_inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.default_rng(77)


def _tmat(m, h):
    return (np.diag(-2.0 * np.ones(m)) + np.diag(np.ones(m - 1), 1) + np.diag(np.ones(m - 1), -1)) / h ** 2


def _op(dim, n, h):
    m = n - 1
    T = _tmat(m, h)
    A1 = T - (h * h / 12.0) * T @ T
    I_ = np.eye(m)
    if dim == 1:
        return A1
    if dim == 2:
        return np.kron(I_, A1) + np.kron(A1, I_)
    return np.kron(np.kron(I_, I_), A1) + np.kron(np.kron(I_, A1), I_) + np.kron(np.kron(A1, I_), I_)


@pytest.mark.parametrize("dim,n", [(1, 8), (2, 6), (3, 5)])
def test_rk4_step_is_taylor_polynomial(orc, dim, n):
    h, a, k = 0.5, 0.7, 0.01
    shape = (n + 1,) * dim
    V = rng.uniform(0, 3, shape)
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    sl = (slice(1, -1),) * dim
    bmask = np.ones(shape, bool)
    bmask[sl] = False
    psi[bmask] = 0
    A = 1j * (a * _op(dim, n, h) - np.diag(V[sl].ravel()))
    x = psi[sl].ravel()
    kA = k * A
    term, acc = x.copy(), x.copy()
    for m in range(1, 5):
        term = kA @ term / m
        acc = acc + term
    out = orc.Problem(dim, n, h, a, 0.0, V).rk4(psi, 1, k)
    np.testing.assert_allclose(out[sl].ravel(), acc, rtol=0, atol=1e-13 * np.abs(acc).max())
    assert np.all(out[bmask] == 0)


def test_single_mode_amplification(orc):
    """Sine mode m on n intervals: eigenvalue of the 1D 2SHOC operator is -(mu/h^2)(1 + mu/12),
    mu = 4 sin^2(pi m / (2n)); one RK4 step multiplies it by R(i k a lambda)."""
    n, h, a = 32, 0.25, 1.3
    i = np.arange(n + 1)
    sym = lambda m: -(4 * math.sin(math.pi * m / (2 * n)) ** 2 / h ** 2) * (1 + math.sin(math.pi * m / (2 * n)) ** 2 / 3)
    k = 0.9 * math.sqrt(8) / (a * abs(sym(n - 1)))      # under the bound for every mode
    for m in (1, 7, 31):
        mode = np.sin(np.pi * m * i / n) + 0j
        mu = 4 * math.sin(math.pi * m / (2 * n)) ** 2
        lam = -(mu / h ** 2) * (1 + mu / 12)
        y = k * a * lam
        R = 1 + 1j * y - y ** 2 / 2 - 1j * y ** 3 / 6 + y ** 4 / 24
        out = orc.Problem(1, n, h, a, 0.0).rk4(mode, 1, k)
        np.testing.assert_allclose(out, R * mode, atol=1e-12)
        assert abs(R) ** 2 == pytest.approx(1 - y ** 6 / 72 + y ** 8 / 576, rel=1e-12)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_linear_bound_closed_form(orc, dim):
    """Eq. kdfull with s = V = 0 and Dirichlet reduces to Eq. kd2shoclin: (3/4) h^2/(d sqrt(2) a)."""
    n, h, a = 8, 0.3, 1.7
    psi = np.zeros((n + 1,) * dim, np.complex128)
    k = orc.Problem(dim, n, h, a, 0.0).max_dt(psi)
    assert k == pytest.approx(0.75 * h * h / (dim * math.sqrt(2) * a), rel=1e-14)


def test_bound_separates_growth(orc):
    """Linear 1D run seeded with the highest mode: grows above the bound, not below it."""
    n, h, a = 64, 0.5, 1.0
    P = orc.Problem(1, n, h, a, 0.0)
    i = np.arange(n + 1)
    psi0 = (np.sin(np.pi * (n - 1) * i / n) + 1e-3 * np.sin(np.pi * i / n)) + 0j
    kmax = P.max_dt(psi0)
    m0 = P.mass(psi0)
    up = P.mass(P.rk4(psi0, 400, 1.05 * kmax))
    down = P.mass(P.rk4(psi0, 400, 0.95 * kmax))
    assert up > 10 * m0
    assert down <= m0 * (1 + 1e-12)


def test_paper_steps_just_below_bound(orc):
    gold = json.load(open(os.path.join(GOLD, "paper_stability_constants.json")))
    for e in gold["paper_k_just_below_bound"]:
        sp = {"fig1": I.paper_fig1, "fig2": I.paper_fig2, "fig3": I.paper_fig3}[e["test"]](e["h"])
        kmax = orc.Problem.from_spec(sp).max_dt(sp.psi0)
        assert e["k"] < kmax < 1.4 * e["k"], (e, kmax)


def test_gvalues_extremes_are_spectral(orc):
    """The extreme G values of Table t:sumresults are 16d/3 and -d/3 (golden fixture)."""
    gold = json.load(open(os.path.join(GOLD, "paper_stability_constants.json")))
    for d in (1, 2, 3):
        G = np.array(gold["G_over_12"][str(d)]) / 12.0
        assert G.max() == pytest.approx(16 * d / 3)
        assert G.min() == pytest.approx(-d / 3)


def test_soliton_bound_value(orc):
    """Config 1: a = s = 1, max|Psi|^2 = 2 at the centre, L_min ~ 0: k_max = sqrt(8) h^2 / (64/12)."""
    sp = I.config_soliton_1d(1024)
    k, aux = orc.Problem.from_spec(sp).max_dt(sp.psi0, return_aux=True)
    h = sp.grid.h
    assert aux[1] == pytest.approx(h * h * 2.0, rel=1e-6)
    assert k == pytest.approx(math.sqrt(8) * h * h / (64 / 12 - aux[0]), rel=1e-14)
    assert k == pytest.approx(0.0050576, abs=2e-7)


def test_msd_bound_uses_boundary_term(orc):
    """MSD adds |B| = (h^2/a)|F_{b-1}/Psi_{b-1}| (Table t:bc2); for a dark soliton with a large phase
    rate this term can dominate."""
    g = I.grid(1, 64, -20, 20)
    (x,) = g.coords()
    psi = I.dark_soliton(x, 0.0, a=1.0, s=-1.0, omega=-200.0, c=0.5)
    P = orc.Problem(1, 64, g.h, 1.0, -1.0, bc="msd")
    k, aux = P.max_dt(psi, return_aux=True)
    assert aux[2] > 0
    m = max(aux[2], 64 / 12 - aux[0], aux[1] + 4 / 12)
    assert k == pytest.approx(math.sqrt(8) * g.h ** 2 / m, rel=1e-14)


def test_mass_semidiscrete_conservation_soliton(orc):
    """The 2SHOC operator is symmetric under Dirichlet 0 and the nonlinearity is a real phase
    rate, so only RK4's O(k^5) local error moves the mass: tiny on the smooth soliton."""
    sp = I.config_soliton_1d(1024)
    P = orc.Problem.from_spec(sp)
    ns, dt = orc.steps_for(10.0, P.max_dt(sp.psi0))
    m0 = P.mass(sp.psi0)
    m1 = P.mass(P.rk4(sp.psi0, ns, dt))
    assert abs(m1 - m0) / m0 < 1e-12


def test_mass_formula(orc):
    """Mass of the bright soliton: integral of 2 sech^2 = 4 (trapezoid on a wide grid)."""
    sp = I.config_soliton_1d(1024)
    assert orc.Problem.from_spec(sp).mass(sp.psi0) == pytest.approx(4.0, rel=1e-10)


@pytest.mark.parametrize("dim", [1, 2])
def test_energy_ground_state(orc, dim):
    """H = -Lap + r^2 (a = 1, s = 0): the Gaussian ground state has energy d * mass;
    the discrete value converges at fourth order in h."""
    errs = []
    for h in (0.5, 0.25):
        sp = I.paper_fig2(h) if dim == 2 else None
        if dim == 1:
            g = I.grid(1, int(12 / h), -6, 6)
            (x,) = g.coords()
            psi = I.gaussian_ho((x,), 0.0)
            P = orc.Problem(1, g.n, h, 1.0, 0.0, x * x)
        else:
            psi, P = sp.psi0, orc.Problem.from_spec(sp)
        errs.append(abs(P.energy(psi) / P.mass(psi) - dim))
    assert errs[1] < errs[0] / 10
    assert errs[1] < 1e-3


def test_energy_conserved_soliton(orc):
    sp = I.config_soliton_1d(1024)
    P = orc.Problem.from_spec(sp)
    e0 = P.energy(sp.psi0)
    e1 = P.energy(P.rk4(sp.psi0, 300, 0.5 * P.max_dt(sp.psi0)))
    assert abs(e1 - e0) < 1e-9 * abs(e0)
    # continuum energy of sqrt(2) sech(x) e^{icx/2} (a = s = 1):
    # int |Psi_x|^2 = int 2 sech^2 tanh^2 + int 2 (c/2)^2 sech^2 = 4/3 + c^2,
    # (s/2) int |Psi|^4 = 2 int sech^4 = 8/3,  so  E = c^2 - 4/3
    # the discrete value converges to it at fourth order in h
    e_half = orc.Problem.from_spec(I.config_soliton_1d(2048)).energy(I.config_soliton_1d(2048).psi0)
    d1, d2 = abs(e0 - (0.25 - 4.0 / 3.0)), abs(e_half - (0.25 - 4.0 / 3.0))
    assert d1 < 2e-5
    assert 12 < d1 / d2 < 20
