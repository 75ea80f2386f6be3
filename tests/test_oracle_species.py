"""Pins of passive-species advection in the oracle.

Species are passive: the hydro part of the state must be bitwise the same
with and without them; a single species with X = 1 keeps rho X = rho bitwise
(its flux is the mass flux times one; several limited species summing to one
do not keep summing to one exactly, since the limiter acts per component);
uniform mass fractions stay uniform;
periodic totals of rho X_s are conserved; and in a uniform flow a smooth
mass fraction is advected exactly like a scalar under 3-D CTU (the same
construction as the entropy-wave pin, with X in place of rho).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import workloads as W
from test_oracle_pins import _scalar_ppm_upwind_faces


def _kh(n=16, nspec=4, seed=5):
    return W.kelvin_helmholtz(n=n, box=n, seed=seed, nspec=nspec)


def test_species_do_not_change_the_hydro():
    with_s = _kh(nspec=4)
    without = _kh(nspec=0)
    A, dA, _ = oracle.run_problem(with_s, 5)
    B, dB, _ = oracle.run_problem(without, 5)
    assert np.array_equal(dA, dB)
    assert np.array_equal(A[:5], B)


def test_unit_mass_fraction_tracks_density_bitwise():
    p = _kh(n=16, nspec=1)
    p.U0 = np.concatenate([p.U0[:5], p.U0[:1]])
    U, _, _ = oracle.run_problem(p, 6)
    assert np.array_equal(U[5], U[0])


def test_species_totals_conserved():
    p = _kh(n=16, nspec=5)
    U, _, cnt = oracle.run_problem(p, 6)
    scale = math.fsum(p.U0[0].ravel())
    for s in range(5):
        assert abs(math.fsum(U[5 + s].ravel()) - math.fsum(p.U0[5 + s].ravel())) <= 1e-13 * scale
    assert not cnt.any()


def test_uniform_mass_fraction_stays_uniform():
    p = _kh(n=16, nspec=2)
    X = [np.full((16, 16, 16), 0.3), np.full((16, 16, 16), 0.7)]
    p.U0 = np.concatenate([p.U0[:5], np.stack([p.U0[0] * X[0], p.U0[0] * X[1]])])
    U, _, _ = oracle.run_problem(p, 6)
    np.testing.assert_allclose(U[5] / U[0], 0.3, rtol=1e-13)
    np.testing.assert_allclose(U[6] / U[0], 0.7, rtol=1e-13)


def test_species_in_uniform_flow_is_scalar_ctu_advection():
    N = 8
    vel = np.array([0.7, 0.4, 0.25])
    x, y, z = W.cell_centres((N, N, N))
    X = 0.5 + 0.3 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * (y + 2 * z))
    U = W.conserved(1.4, 1.3, vel[0], vel[1], vel[2], 1.0, [X])
    dx = 1.0 / N
    dt = 0.4 * dx
    P = oracle.make_params(1.4, (dx,) * 3, nspec=1)
    G = oracle.fill_domain(oracle.grow(U), P)
    Gn, cnt = oracle.advance_box(G, P, dt)
    Un = oracle.valid(Gn)
    got = Un[5] / Un[0]
    ax = {0: 2, 1: 1, 2: 0}
    nu = vel * dt / dx
    face = {d: _scalar_ppm_upwind_faces(X, ax[d], nu[d]) for d in range(3)}
    flux = {d: vel[d] * face[d] for d in range(3)}
    diff = lambda f, d: np.roll(f, 0, ax[d]) - np.roll(f, 1, ax[d])
    f1 = {}
    for a in range(3):
        for b in range(3):
            if a != b:
                f1[(a, b)] = vel[a] * (face[a] - dt / (3 * dx) * diff(flux[b], b))
    fin = {}
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        fin[a] = vel[a] * (face[a] - dt / (2 * dx) * diff(f1[(b, c)], b) - dt / (2 * dx) * diff(f1[(c, b)], c))
    want = X - dt / dx * (diff(fin[0], 0) + diff(fin[1], 1) + diff(fin[2], 2))
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-13)
    np.testing.assert_allclose(Un[0], 1.3, rtol=1e-14)
