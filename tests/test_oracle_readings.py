"""Pins of three readings of the oracle that the broader pins leave open: the
two-level time step, passive species at reflecting walls, and the flattening
tie.  Each is checked against a value computed here from the definition
(numpy signal speeds, a hand-worked pressure stencil) or against an
invariant (impermeable walls conserve every species), so that a plausible
mistake in the oracle -- the factor 2 of the fine level's CFL limit dropped,
min taken as max, species mishandled in the wall's ghost cells, the opposite
side taken on a pressure tie -- fails one of them.

Species in the mirrored outside state of a wall face are a reading that cannot
change any result: the ghost side already traces the mirror's species to the
wall face, bitwise (asserted below), so an oracle that left species out of the
mirror gives bitwise the same run."""
import math

import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import workloads as W

NG = oracle.NG


def _speed(U, gamma, dx):
    """max over cells of max_d (|u_d| + c) / dx_d of a conserved state (5+, nz, ny, nx)."""
    rho = U[0]
    vel = [U[1] / rho, U[2] / rho, U[3] / rho]
    ke = 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    p = (gamma - 1.0) * (U[4] - ke)
    c = np.sqrt(gamma * p / rho)
    return max(float(((np.abs(vel[d]) + c) / dx[d]).max()) for d in range(3))


def _two_level_case(fast_on_fine: bool):
    """Coarse 24^3 periodic, fine patch over coarse cells 8..15 (fine 16^3); a
    uniform slow state with one fast cell, on the fine patch or on the coarse
    level outside it."""
    gamma, n = 1.4, 24
    clo, chi = np.array([8, 8, 8]), np.array([15, 15, 15])
    Uc = W.conserved(gamma, np.ones((n, n, n)), 0.1, 0.0, 0.0, np.ones((n, n, n)))
    nf = 2 * (chi - clo + 1)
    Uf = W.conserved(gamma, np.ones(tuple(nf[::-1])), 0.1, 0.0, 0.0, np.ones(tuple(nf[::-1])))
    if fast_on_fine:
        Uf[1, 5, 6, 7] = 2.5 * Uf[0, 5, 6, 7]  # u_x = 2.5 in one fine cell
        Uf[4, 5, 6, 7] = 1.0 / (gamma - 1.0) + 0.5 * 2.5 ** 2
    else:
        Uc[2, 2, 3, 20] = -1.8 * Uc[0, 2, 3, 20]  # u_y = -1.8 in one uncovered coarse cell
        Uc[4, 2, 3, 20] = 1.0 / (gamma - 1.0) + 0.5 * 1.8 ** 2
    dx = (1.0 / n,) * 3
    Pc = oracle.make_params(gamma, dx, cfl=0.5)
    Pf = oracle.with_faces(oracle.make_params(gamma, tuple(v / 2 for v in dx), cfl=0.5), (-(1 << 30),) * 3,
                           (-(1 << 30),) * 3)
    return Uc, Uf, clo, chi, Pc, Pf, gamma, dx


@pytest.mark.parametrize("fast_on_fine", [True, False])
def test_two_level_dt_takes_the_binding_level(fast_on_fine):
    """dt_c = min(cfl / s_c, 2 (cfl / s_f)): the fine substep (dt_c / 2) meets
    the fine level's CFL limit and the coarse step the coarse one, with
    equality on the level that holds the fastest signal (section 3.2:
    subcycled levels, each with its own CFL-limited step)."""
    Uc, Uf, clo, chi, Pc, Pf, gamma, dx = _two_level_case(fast_on_fine)
    s_c = _speed(Uc, gamma, dx)
    s_f = _speed(Uf, gamma, tuple(v / 2 for v in dx))
    _, _, dt_c, cnt = oracle.two_level_step(oracle.grow(Uc), oracle.grow(Uf), clo, chi, Pc, Pf)
    assert not cnt.any()
    cfl = Pc.cfl
    if fast_on_fine:
        assert s_f > 2.0 * s_c  # the fine level binds
        assert dt_c == pytest.approx(2.0 * cfl / s_f, rel=1e-14)
        assert (0.5 * dt_c) * s_f == pytest.approx(cfl, rel=1e-14)
        assert dt_c * s_c < 0.75 * cfl
    else:
        assert s_c > 0.5 * s_f  # the coarse level binds
        assert dt_c == pytest.approx(cfl / s_c, rel=1e-14)
        assert dt_c * s_c == pytest.approx(cfl, rel=1e-14)
        assert (0.5 * dt_c) * s_f < 0.75 * cfl


def test_species_at_reflecting_walls_are_conserved_and_not_transported():
    """Walled Rayleigh-Taylor with two species: the walls let no species
    through (every species total conserved over 60 steps to round-off), and the
    species fluxes on the wall faces -- normal, both first-stage corrections and
    final -- are zero to round-off."""
    prob = W.rayleigh_taylor(n=(12, 8, 24), seed=7, boxes=[((0, 0, 0), (11, 7, 23))], nspec=2)
    U, _, cnt = oracle.run_problem(prob, 60)
    assert not cnt.any()
    for m in (0, 5, 6):
        t0, t1 = math.fsum(prob.U0[m].ravel()), math.fsum(U[m].ravel())
        assert abs(t1 - t0) <= 1e-13 * abs(t0), (m, t0, t1)
    # one step of a state that has moved: species fluxes on the two z walls
    P = oracle.params_of(prob)
    G = oracle.fill_domain(oracle.grow(U), P)
    dt = P.cfl / oracle.signal_speed(G, P)
    _, _, st = oracle.advance_box(G, P, dt, stages=True)
    nz = prob.n[2]
    scale = float(np.abs(U[0]).max()) * math.sqrt(1.4 * 3.0)
    for key in ("fn2", "ff2", "f14", "f15"):
        for face in (0, nz):
            f = st[key][5:7, face + 1, 1:-1, 1:-1]
            f = f[np.isfinite(f)]
            assert f.size and np.abs(f).max() <= 1e-15 * scale, (key, face, float(np.abs(f).max()))
    # the interior z faces do carry species (the pin is not vacuous)
    assert np.abs(st["ff2"][5, nz // 2 + 1, 1:-1, 1:-1]).max() > 1e-8
    # why the species of the mirrored outside state cannot change a result: the
    # ghost cells mirror the interior and species trace with the normal
    # velocity, so the species the ghost side traces to a wall face already
    # equal (bitwise) the inside state's, which the mirror copies
    for face in (0, nz):
        left, right = st["ql2"][5:7, face + 1, 1:-1, 1:-1], st["qr2"][5:7, face + 1, 1:-1, 1:-1]
        assert np.array_equal(left, right), face


def test_flattening_tie_takes_the_upper_neighbour():
    """CW84 flattening: phi_i = 1 - max(f~_i, f~_{i-s}) with s the sign of
    p_{i+1} - p_{i-1}; on a tie (p_{i+1} = p_{i-1}) s = -1, so the upper
    neighbour's shock indicator counts.  Hand-worked stencil along x around
    cell c: p = (1, 1, 1, 1, 2, 2.25) at c-2..c+3 and a compression u_c > u_{c+2}
    make cell c+1 a shock with f~ = 10 (1 / 1.25 - 0.75) = 0.5, cells c-1 and
    c none; so phi_c = 0.5 (s = +1 would give 1)."""
    gamma, nx = 1.4, 16
    c = 7
    p = np.ones(nx)
    p[c + 2] = 2.0
    p[c + 3:] = 2.25
    u = np.zeros(nx)
    u[c] = 0.5
    shape = (4, 4, nx)
    rho = np.ones(shape)
    P3 = np.broadcast_to(p, shape).copy()
    U3 = np.broadcast_to(u, shape).copy()
    U0 = W.conserved(gamma, rho, U3, 0.0, 0.0, P3)
    P = oracle.make_params(gamma, (1.0 / nx, 0.25, 0.25), bc_lo=(1, 0, 0), bc_hi=(1, 0, 0))
    G = oracle.fill_domain(oracle.grow(U0), P)
    _, _, st = oracle.advance_box(G, P, 1e-6, stages=True)
    phi = st["phi"][0, 1:-1, 1:-1, 1:-1]  # cells 0..n-1
    # hand values: f~_{c+1} = 10 (|dp1| / |dp2| - 0.75) with dp1 = p_{c+2} - p_c = 1, dp2 = p_{c+3} - p_{c-1} = 1.25
    assert np.all(np.abs(phi[:, :, c] - 0.5) <= 1e-14), phi[:, :, c]
    assert np.all(np.abs(phi[:, :, c + 1] - 0.5) <= 1e-14)   # the shocked cell itself
    assert np.all(phi[:, :, c - 1] == 1.0)                   # neither it nor c-2 is shocked
