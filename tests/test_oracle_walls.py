"""Pins of the oracle's reflecting walls: a solid wall lets no mass (and no
tangential momentum) through, so a closed direction conserves them to round-off
even under gravity, and the fluxes on the wall faces carry no mass.  Without
the mirrored outside state the gravity predictor (+dt/2 g on both sides of the
wall face) breaks the symmetry of the wall's Riemann problem and mass leaks
through the wall at a rate far above round-off."""
import math

import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import workloads as W


def _totals(U):
    return [math.fsum(U[m].ravel()) for m in range(U.shape[0])]


@pytest.mark.parametrize("riemann,limiter", [(0, 0), (1, 0), (0, 1)])
def test_mass_and_tangential_momentum_conserved_between_walls_under_gravity(riemann, limiter):
    prob = W.rayleigh_taylor(n=(16, 8, 32), seed=3, boxes=[((0, 0, 0), (15, 7, 31))])
    prob.riemann, prob.limiter = riemann, limiter
    U, _, cnt = oracle.run_problem(prob, 60)
    assert not cnt.any()
    t0, t1 = _totals(prob.U0), _totals(U)
    mass = t0[0]
    scale = math.fsum(np.abs(prob.U0[4]).ravel())
    assert abs(t1[0] - t0[0]) <= 1e-13 * mass, (t0[0], t1[0])
    for m in (1, 2):  # x, y momentum: periodic directions and tangential at the z walls
        assert abs(t1[m] - t0[m]) <= 1e-13 * scale, (m, t0[m], t1[m])


def test_wall_faces_carry_no_mass():
    prob = W.rayleigh_taylor(n=(8, 8, 16), seed=5, boxes=[((0, 0, 0), (7, 7, 15))])
    P = oracle.params_of(prob)
    G = oracle.fill_domain(oracle.grow(prob.U0), P)
    dt = P.cfl / oracle.signal_speed(G, P)
    _, _, st = oracle.advance_box(G, P, dt, stages=True)
    nz = prob.n[2]
    flux_scale = float(np.abs(prob.U0[0]).max()) * math.sqrt(1.4 * 2.5)
    for key in ("fn2", "ff2"):
        for face in (0, nz):
            f = st[key][0, face + 1, 1:-1, 1:-1]  # mass flux on the wall face, interior x, y
            assert np.abs(f).max() <= 1e-15 * flux_scale, (key, face, float(np.abs(f).max()))
    for p in (4, 5):  # stage-1 fluxes of the z faces
        f = st[f"f1{p}"][0, [1, nz + 1]][:, 1:-1, 1:-1]
        assert np.abs(f[np.isfinite(f)]).max() <= 1e-15 * flux_scale


def test_method_of_lines_walls_conserve_mass():
    prob = W.rayleigh_taylor(n=(16, 8, 32), seed=4, boxes=[((0, 0, 0), (15, 7, 31))])
    prob.scheme = 1
    U, _, cnt = oracle.run_problem(prob, 40)
    assert not cnt.any()
    m0, m1 = math.fsum(prob.U0[0].ravel()), math.fsum(U[0].ravel())
    assert abs(m1 - m0) <= 1e-13 * m0


def test_closed_box_conserves_mass_and_energy_without_gravity():
    nn = (24, 6, 6)
    x, y, z = W.cell_centres(nn)
    rho = np.where(x < 0.4, 1.0, 0.125)
    p = np.where(x < 0.4, 1.0, 0.1)
    U0 = W.conserved(1.4, rho, 0.3, 0.0, 0.0, p)
    prob = W.Problem("box", nn, 1.4, U0, [((0, 0, 0), (23, 5, 5))], (W.BC_REFLECT, 0, 0), (W.BC_REFLECT, 0, 0))
    U, _, cnt = oracle.run_problem(prob, 80)
    assert not cnt.any()
    t0, t1 = _totals(U0), _totals(U)
    for m in (0, 4):
        assert abs(t1[m] - t0[m]) <= 1e-13 * abs(t0[m]), (m, t0[m], t1[m])
