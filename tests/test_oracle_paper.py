"""The oracle reproduces the paper's printed accuracy tables (Sec. 4, Figs. 1-3) and the
exact-solution behaviour of the 1D bright soliton.

Figs. 2 and 3 are reproduced to every printed digit on [-6, 6]^d (the paper's domain
rule: exact solution ~ sqrt(eps) on the boundary).  Fig. 1's domain is not stated; the
symmetric [-28.25, 28.25] is assumed and compared to within 1% / 0.003 in the order.
"""
import json
import os

import numpy as np
import pytest

import nlse_inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    return json.load(open(os.path.join(GOLD, name)))


def run_paper(orc, spec, lap, exact):
    P = orc.Problem.from_spec(spec, lap)
    er, ei, _ = orc.paper_error(P, spec.psi0, exact, spec.t_end, spec.steps)
    return er, ei


def sig5(x):
    return float(f"{x:.5g}")


@pytest.mark.parametrize("hi", [0, 1, 2])
def test_fig2_digits(orc, hi):
    g = gold("paper_fig2_gaussian_2d.json")
    h = g["h"][hi]
    sp = I.paper_fig2(h)
    c = sp.grid.coords()
    ex = lambda t: I.gaussian_ho(c, t)
    er, ei = run_paper(orc, sp, "2shoc", ex)
    assert (sig5(er), sig5(ei)) == (g["shoc_error_real"][hi], g["shoc_error_imag"][hi])
    cr, ci = run_paper(orc, sp, "cd", ex)
    assert (sig5(cr), sig5(ci)) == (g["cd_error_real"][hi], g["cd_error_imag"][hi])


def test_fig3_digits_h1(orc):
    g = gold("paper_fig3_gaussian_3d.json")
    sp = I.paper_fig3(1.0)
    c = sp.grid.coords()
    ex = lambda t: I.gaussian_ho(c, t)
    er, ei = run_paper(orc, sp, "2shoc", ex)
    assert (sig5(er), sig5(ei)) == (g["shoc_error_real"][0], g["shoc_error_imag"][0])
    cr, ci = run_paper(orc, sp, "cd", ex)
    assert (sig5(cr), sig5(ci)) == (g["cd_error_real"][0], g["cd_error_imag"][0])


@pytest.mark.slow
def test_fig3_digits_h_half(orc):
    g = gold("paper_fig3_gaussian_3d.json")
    sp = I.paper_fig3(0.5)
    c = sp.grid.coords()
    er, ei = run_paper(orc, sp, "2shoc", lambda t: I.gaussian_ho(c, t))
    assert (sig5(er), sig5(ei)) == (g["shoc_error_real"][1], g["shoc_error_imag"][1])


def test_fig1_msd_dark_soliton(orc):
    g = gold("paper_fig1_dark_soliton_msd.json")
    errs = []
    for hi in range(3):
        h = g["h"][hi]
        sp = I.paper_fig1(h)
        (x,) = sp.grid.coords()
        er, ei = run_paper(orc, sp, "2shoc", lambda t: I.dark_soliton(x, t))
        assert er == pytest.approx(g["shoc_error_real"][hi], rel=0.01)
        assert ei == pytest.approx(g["shoc_error_imag"][hi], rel=0.01)
        errs.append((er, ei))
    for hi in (1, 2):
        o_r = orc.order(errs[hi - 1][0], errs[hi][0], g["h"][hi - 1], g["h"][hi])
        o_i = orc.order(errs[hi - 1][1], errs[hi][1], g["h"][hi - 1], g["h"][hi])
        assert o_r == pytest.approx(g["shoc_order_real"][hi], abs=0.003)
        assert o_i == pytest.approx(g["shoc_order_imag"][hi], abs=0.003)


def test_fig1_cd_second_order(orc):
    g = gold("paper_fig1_dark_soliton_msd.json")
    sp = I.paper_fig1(0.5)
    (x,) = sp.grid.coords()
    er, ei = run_paper(orc, sp, "cd", lambda t: I.dark_soliton(x, t))
    assert er == pytest.approx(g["cd_error_real"][0], rel=0.01)
    assert ei == pytest.approx(g["cd_error_imag"][0], rel=0.01)


def test_bright_soliton_fourth_order(orc):
    """1D bright soliton (a = s = 1, eta = 1, c = 0.5) on [-50, 50] to t = 10 at dt = 0.5 k_max:
    relative L2 error against the exact solution falls ~16x per halving of h."""
    errs = {}
    for n in (512, 1024, 2048):
        sp = I.config_soliton_1d(n)
        P = orc.Problem.from_spec(sp)
        ns, dt = orc.steps_for(10.0, P.max_dt(sp.psi0))
        psi = P.rk4(sp.psi0, ns, dt)
        (x,) = sp.grid.coords()
        errs[n] = orc.rel_l2(psi, I.bright_soliton(x, 10.0, 1.0, 1.0, 1.0, 0.5))
    assert errs[1024] == pytest.approx(1.31e-4, rel=0.02)
    o1 = np.log2(errs[512] / errs[1024])
    o2 = np.log2(errs[1024] / errs[2048])
    assert 3.9 < o1 < 4.1 and 3.9 < o2 < 4.1
