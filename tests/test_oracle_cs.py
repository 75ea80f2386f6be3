"""Pins of the oracle's extremum-preserving PPM limiter (Colella & Sekora 2008).

What the mathematics fixes: cell averages of a quadratic with an extremum are
reconstructed exactly (CW84's limiter flattens that cell, CS08 keeps it), the
fourth-order interface value is exact for a cubic in a monotone region,
parabolas next to a jump stay inside the neighbouring averages, and a smooth
advected wave converges at second order in the maximum norm, where CW84's
clipping of smooth extrema holds it near 1.5.  Plus Sod against the exact
solution and conservation with the limiter in the full step.
"""
import math

import numpy as np
import pytest

import exact_riemann as ER
import oracle
from paper_1711_06203_amd import workloads as W


def _averages(F, x0, h, k):
    """Cell averages of a function with antiderivative F over cells k."""
    return np.array([(F(x0 + (i + 1) * h) - F(x0 + i * h)) / h for i in k])


@pytest.mark.parametrize("x0", [-2.5, -2.2, -2.8])
def test_quadratic_extremum_is_reconstructed_exactly(x0):
    # q(x) = 1 - x^2, antiderivative x - x^3/3; the middle cell holds the maximum
    h = 1.0
    F = lambda x: x - x ** 3 / 3.0
    a = _averages(F, x0, h, range(5))
    out = oracle.ppm_cell(a, 1.0, limiter=1)
    xl, xr = x0 + 2 * h, x0 + 3 * h
    np.testing.assert_allclose(out[:2], [1 - xl ** 2, 1 - xr ** 2], rtol=0, atol=1e-14)
    # the parabola's mean is the cell average
    assert out[0] + 0.5 * out[2] + out[3] / 6.0 == pytest.approx(a[2], abs=1e-14)
    cw = oracle.ppm_cell(a, 1.0, limiter=0)
    assert cw[0] == cw[1] == a[2]  # CW84 flattens the extremum cell


def test_cubic_in_a_monotone_region_gives_exact_interfaces():
    # c(x) = x^3 + x on cells [0.1 + i h]: monotone, gentle curvature
    h = 0.05
    F = lambda x: x ** 4 / 4.0 + x ** 2 / 2.0
    a = _averages(F, 0.1, h, range(5))
    out = oracle.ppm_cell(a, 1.0, limiter=1)
    xl, xr = 0.1 + 2 * h, 0.1 + 3 * h
    np.testing.assert_allclose(out[:2], [xl ** 3 + xl, xr ** 3 + xr], rtol=0, atol=1e-14)


@pytest.mark.parametrize("a", [(0, 0, 0, 1, 1), (0, 0, 1, 1, 1), (1, 1, 1, 0, 0), (0, 0, 0.5, 1, 1), (2, 2, 1.2, 1, 1)])
def test_parabola_next_to_a_jump_stays_bounded(a):
    a = np.asarray(a, dtype=float)
    aL, aR, da, a6 = oracle.ppm_cell(a, 1.0, limiter=1)
    lo, hi = min(a[1:4]), max(a[1:4])
    x = np.linspace(0.0, 1.0, 201)
    vals = aL + x * (da + a6 * (1.0 - x))
    assert vals.min() >= lo - 1e-14 and vals.max() <= hi + 1e-14


def _wave_orders(limiter, scheme):
    errs = []
    T = 1.0 / 3.0
    for N in (32, 64, 128):
        nn = (N, 4, 4)
        x, y, z = W.cell_centres(nn)
        U0 = W.conserved(1.4, 1.0 + 0.2 * np.sin(2 * np.pi * x), 1.0, 0.0, 0.0, 1.0)
        prob = W.Problem("wave1d", nn, 1.4, U0, [((0, 0, 0), (N - 1, 3, 3))], scheme=scheme, limiter=limiter)
        c = math.sqrt(1.4 / 0.8)
        ns = int(math.ceil(T / (0.4 / ((1 + c) * N))))
        U, _, cnt = oracle.run(U0, oracle.params_of(prob), ns, dt_fixed=T / ns)
        assert not cnt.any()
        # exact cell averages of the advected wave
        ex = 1.0 + 0.2 * (np.cos(2 * np.pi * (x - 0.5 / N - T)) - np.cos(2 * np.pi * (x + 0.5 / N - T))) / (2 * np.pi / N)
        errs.append(np.abs(U[0] - ex).max())
    return [math.log2(errs[i] / errs[i + 1]) for i in range(2)], errs


@pytest.mark.parametrize("scheme", [0, 1])
def test_smooth_extrema_converge_at_second_order_in_max_norm(scheme):
    cs, ecs = _wave_orders(1, scheme)
    cw, ecw = _wave_orders(0, scheme)
    assert min(cs) >= 1.9, (cs, ecs)
    assert min(cw) < 1.75, (cw, ecw)         # CW84 clips the smooth extrema
    assert ecs[-1] < 0.5 * ecw[-1]


def test_sod_with_the_cs_limiter():
    for scheme in (0, 1):
        errs = []
        for N in (64, 128):
            prob = W.sod(n=(N, 4, 4))
            prob.limiter = 1
            prob.scheme = scheme
            P = oracle.params_of(prob)
            U, t = prob.U0, 0.0
            while t < 0.2 - 1e-14:
                G = oracle.fill_domain(oracle.grow(U), P)
                dt = min(P.cfl / oracle.signal_speed(G, P), 0.2 - t)
                U, _, cnt = oracle.run(U, P, 1, dt_fixed=dt)
                assert not cnt.any()
                t += dt
            x = (np.arange(N) + 0.5) / N
            ex = ER.cell_average(x - 0.5 / N, x + 0.5 / N, 0.2, 0.5, (1, 0, 1), (0.125, 0, 0.1))
            errs.append(np.abs(U[0, 1, 1] - ex).mean())
        assert errs[1] < 3.5e-3 and errs[0] / errs[1] > 1.6, errs


def test_cs_conservation_and_uniform_state():
    prob = W.kelvin_helmholtz(n=16, box=16, seed=6, nspec=1)
    prob.limiter = 1
    U, _, cnt = oracle.run(prob.U0, oracle.params_of(prob), 4)
    for m in range(U.shape[0]):
        t0, t1 = math.fsum(prob.U0[m].ravel()), math.fsum(U[m].ravel())
        scale = max(math.fsum(np.abs(prob.U0[m]).ravel()), math.fsum(prob.U0[0].ravel()))
        assert abs(t1 - t0) <= 1e-13 * scale
    assert not cnt.any()
    uni = W.uniform(n=(8, 6, 5))
    uni.limiter = 1
    Uu, _, _ = oracle.run(uni.U0, oracle.params_of(uni), 3)
    for m in range(5):
        assert np.all(Uu[m] == uni.U0[m][0, 0, 0])


def test_parabola_is_monotone_where_the_averages_are():
    """Away from extrema the overshoot correction leaves a parabola with no
    interior extremum (CW84's condition): monotone averages give a monotone
    parabola across the cell."""
    rng = np.random.default_rng(12)
    x = np.linspace(0.0, 1.0, 401)
    for _ in range(400):
        a = np.cumsum(rng.exponential(1.0, 5) ** 3)
        if rng.random() < 0.5:
            a = a[::-1].copy()
        aL, aR, da, a6 = oracle.ppm_cell(a, 1.0, limiter=1)
        v = aL + x * (da + a6 * (1.0 - x))
        dv = np.diff(v) * np.sign(a[4] - a[0])
        assert dv.min() >= -1e-12 * max(1.0, abs(a).max()), a
