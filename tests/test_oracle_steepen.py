"""Pins of the oracle's CW84 contact steepening (density only, CW84 limiter).

Properties the method is built for: an advected contact stays within about
two zones (without steepening it spreads to six in the same run), the
steepening switches itself off for a jump that carries a pressure jump of the
same size (a shock) and for smooth data (the solution is then bitwise the
unsteepened one), and a fully steepened parabola is steeper and stays within
its neighbours; plus Sod against the exact solution (the contact error drops)
and conservation.
"""
import math

import numpy as np
import pytest

import exact_riemann as ER
import oracle
from paper_1711_06203_amd import workloads as W


def _contact(N, steepen, steps):
    nn = (N, 2, 2)
    x, y, z = W.cell_centres(nn)
    rho = np.where(np.abs(x - 0.3) < 0.15, 1.0, 0.125)
    U0 = W.conserved(1.4, rho, 1.0, 0.0, 0.0, 1.0)
    prob = W.Problem("contact", nn, 1.4, U0, [((0, 0, 0), (N - 1, 1, 1))], steepen=steepen)
    U, dts, cnt = oracle.run(U0, oracle.params_of(prob), steps)
    assert not cnt.any()
    return U, dts.sum(), x


def test_an_advected_contact_stays_sharp():
    Us, T, x = _contact(64, 1, 100)
    Un, _, _ = _contact(64, 0, 100)
    f = lambda U: (U[0, 0, 0] - 0.125) / 0.875
    mid_s = int(((f(Us) > 0.05) & (f(Us) < 0.95)).sum())
    mid_n = int(((f(Un) > 0.05) & (f(Un) < 0.95)).sum())
    assert mid_s <= 2 and mid_n >= 5, (mid_s, mid_n)
    # closer to the exactly translated profile
    xx = (x[0, 0] - T) % 1.0
    exact = np.where(np.abs(xx - 0.3) < 0.15, 1.0, 0.125)
    assert np.abs(Us[0, 0, 0] - exact).mean() < 0.85 * np.abs(Un[0, 0, 0] - exact).mean()


def test_a_jump_with_a_pressure_jump_is_not_steepened():
    r = (1.0, 0.95, 0.5625, 0.175, 0.125)
    assert oracle.steep_eta(r, 1.0, 1.0, 1.4) == 1.0       # contact: full weight
    assert oracle.steep_eta(r, 1.0, 0.4, 1.4) == 0.0       # pressure jumps too: a shock
    a = np.array(r)
    np.testing.assert_array_equal(oracle.ppm_cell(a, 1.0, 0, 0.0), oracle.ppm_cell(a, 1.0))


def test_a_steepened_parabola_is_steeper_and_bounded():
    a = np.array((1.0, 0.95, 0.5625, 0.175, 0.125))
    plain = oracle.ppm_cell(a, 1.0, 0, 0.0)
    steep = oracle.ppm_cell(a, 1.0, 0, 1.0)
    assert abs(steep[2]) > abs(plain[2])
    x = np.linspace(0.0, 1.0, 201)
    v = steep[0] + x * (steep[2] + steep[3] * (1.0 - x))
    assert v.min() >= a[3] - 1e-14 and v.max() <= a[1] + 1e-14


def test_smooth_flow_is_not_steepened():
    """A resolved smooth wave (entropy wave with 32+ cells per wavelength, with
    a pressure-free density variation that would qualify as a contact) has no
    inflection sharp enough for the detector: bitwise the unsteepened run."""
    for N in (32, 64):
        nn = (N, 4, 4)
        x, y, z = W.cell_centres(nn)
        U0 = W.conserved(1.4, 1.0 + 0.2 * np.sin(2 * np.pi * x), 1.0, 0.0, 0.0, 1.0)
        runs = []
        for st in (0, 1):
            prob = W.Problem("wave", nn, 1.4, U0, [((0, 0, 0), (N - 1, 3, 3))], steepen=st)
            runs.append(oracle.run(U0, oracle.params_of(prob), 6)[0])
        assert np.array_equal(runs[0], runs[1])


def test_sod_contact_error_drops():
    errs = {}
    for st in (0, 1):
        prob = W.sod(n=(128, 4, 4))
        prob.steepen = st
        P = oracle.params_of(prob)
        U, t = prob.U0, 0.0
        while t < 0.2 - 1e-14:
            G = oracle.fill_domain(oracle.grow(U), P)
            dt = min(P.cfl / oracle.signal_speed(G, P), 0.2 - t)
            U, _, cnt = oracle.run(U, P, 1, dt_fixed=dt)
            assert not cnt.any()
            t += dt
        x = (np.arange(128) + 0.5) / 128
        ex = ER.cell_average(x - 0.5 / 128, x + 0.5 / 128, 0.2, 0.5, (1, 0, 1), (0.125, 0, 0.1))
        errs[st] = np.abs(U[0, 1, 1] - ex).mean()
    assert errs[1] < errs[0] and errs[1] < 3e-3, errs


def test_steepening_conserves():
    prob = W.kelvin_helmholtz(n=16, box=16, seed=8)
    prob.steepen = 1
    U, _, cnt = oracle.run(prob.U0, oracle.params_of(prob), 4)
    for m in range(5):
        t0, t1 = math.fsum(prob.U0[m].ravel()), math.fsum(U[m].ravel())
        scale = max(math.fsum(np.abs(prob.U0[m]).ravel()), math.fsum(prob.U0[0].ravel()))
        assert abs(t1 - t0) <= 1e-13 * scale
    assert not cnt.any()


def test_only_the_density_is_steepened():
    """One step's traced face states with and without steepening: every
    component but the density is bitwise the same, the density's differ
    around the contact."""
    N = 32
    nn = (N, 4, 4)
    x, y, z = W.cell_centres(nn)
    inside = np.abs(x - 0.4) < 0.2
    U0 = W.conserved(1.4, np.where(inside, 1.0, 0.125), 0.5, np.where(inside, 0.3, -0.2), 0.1, 1.0,
                     [np.where(inside, 0.9, 0.1)])
    U0, _, _ = oracle.run(U0, oracle.make_params(1.4, (1.0 / N, 0.25, 0.25), nspec=1), 3)  # smear it
    st = {}
    for s_ in (0, 1):
        P = oracle.make_params(1.4, (1.0 / N, 0.25, 0.25), nspec=1, steepen=s_)
        G = oracle.fill_domain(oracle.grow(U0), P)
        _, _, st[s_] = oracle.advance_box(G, P, 0.2 / N, stages=True)
    for key in ("ql0", "qr0"):
        a, b = st[0][key], st[1][key]
        np.testing.assert_array_equal(a[1:], b[1:])
        assert not np.array_equal(a[0], b[0])
