"""Pins of the oracle's two-level (subcycled, refluxed) step.

Closed forms and invariants: interpolation of a linear coarse field gives the
fine cell averages exactly; a uniform state stays bitwise uniform (fluxes
equal on both levels, register zero); composite totals are conserved to
round-off on a periodic domain; a smooth wave on the fine patch tracks a
single-level fine-resolution run much more closely than the coarse run does.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import workloads as W


def _two_level_problem(n=24, patch=((8, 8, 8), (16, 16, 16)), field=None, vel=(1.0, 0.5, 0.25)):
    clo, chi = patch
    x, y, z = W.cell_centres((n, n, n))
    f = field or (lambda x, y, z: 1.0 + 0.2 * np.sin(2 * np.pi * (x + y + z)))
    p = W.Problem("tl", (n, n, n), 1.4, W.conserved(1.4, f(x, y, z), *vel, 1.0),
                  W.regular_boxes((n, n, n), (n // 2,) * 3))
    flo = tuple(2 * c for c in clo)
    nf = tuple(2 * (chi[d] - clo[d]) for d in range(3))
    axes = [(np.arange(flo[d], flo[d] + nf[d]) + 0.5) / (2 * n) for d in range(3)]
    zf, yf, xf = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    p.U0_fine = W.conserved(1.4, f(xf, yf, zf), *vel, 1.0)
    p.fine_lo = flo
    p.fine_boxes = W.regular_boxes(nf, (8, 8, 8), origin=flo)
    return p


def test_cf_interp_linear_is_exact():
    rng = np.random.default_rng(4)
    g = rng.uniform(-1, 1, (5, 3))
    c0 = rng.uniform(1, 2, 5)
    lo = np.array([3, 5, 7])
    shape = (6, 6, 6)
    k, j, i = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    X = np.stack([i + lo[0] + 0.5, j + lo[1] + 0.5, k + lo[2] + 0.5])
    Uc = np.stack([c0[m] + g[m, 0] * X[0] + g[m, 1] * X[1] + g[m, 2] * X[2] for m in range(5)])
    fine = np.array([[2 * (lo[0] + a) + p, 2 * (lo[1] + b) + q, 2 * (lo[2] + c) + r]
                     for a in (1, 2, 3) for b in (1, 4) for c in (2, 3) for p in (0, 1) for q in (0, 1) for r in (0, 1)])
    got = oracle.cf_interp(Uc, lo, fine)
    centre = (fine + 0.5) / 2.0          # fine cell centres in coarse units
    want = np.stack([c0[m] + g[m] @ centre.T for m in range(5)])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_two_level_uniform_state_bitwise():
    p = _two_level_problem(field=lambda x, y, z: np.full_like(x, 1.3), vel=(0.3, -0.2, 0.1))
    Uc, Uf, dts, cnt = oracle.run_two_level(p, 3)
    for m in range(5):
        assert np.all(Uc[m] == p.U0[m].flat[0])
        assert np.all(Uf[m] == p.U0_fine[m].flat[0])
    assert not cnt.any()


def test_two_level_composite_conservation():
    p = _two_level_problem()
    t0 = [math.fsum(p.U0[m].ravel()) for m in range(5)]
    Uc, Uf, dts, cnt = oracle.run_two_level(p, 5)
    scale = math.fsum(np.abs(p.U0[0]).ravel())
    for m in range(5):
        assert abs(math.fsum(Uc[m].ravel()) - t0[m]) <= 1e-13 * scale
    # covered coarse cells are the average of their children
    flo = np.array(p.fine_lo)
    clo = flo // 2
    nf = np.array(Uf.shape[1:][::-1])
    cov = Uc[:, clo[2]:clo[2] + nf[2] // 2, clo[1]:clo[1] + nf[1] // 2, clo[0]:clo[0] + nf[0] // 2]
    avg = Uf.reshape(5, nf[2] // 2, 2, nf[1] // 2, 2, nf[0] // 2, 2).mean(axis=(2, 4, 6))
    np.testing.assert_allclose(cov, avg, rtol=1e-14, atol=1e-15)


def test_fine_patch_tracks_fine_resolution_run():
    n = 24
    p = _two_level_problem(n=n)
    steps = 4
    Uc, Uf, dts, _ = oracle.run_two_level(p, steps)
    # single-level run at fine resolution with the fine substeps' dt
    pf = W.smooth_wave(n=2 * n)
    pf.U0 = W.conserved(1.4, 1.0 + 0.2 * np.sin(2 * np.pi * sum(W.cell_centres((2 * n,) * 3))), 1.0, 0.5, 0.25, 1.0)
    Gf = oracle.grow(pf.U0)
    Pf = oracle.params_of(pf)
    for dt in dts:
        for _ in range(2):
            oracle.fill_domain(Gf, Pf)
            Gf, _ = oracle.advance_box(Gf, Pf, 0.5 * dt)
    ref = oracle.valid(Gf)
    flo = np.array(p.fine_lo)
    nf = np.array(Uf.shape[1:][::-1])
    ref_patch = ref[:, flo[2]:flo[2] + nf[2], flo[1]:flo[1] + nf[1], flo[0]:flo[0] + nf[0]]
    # coarse-only run with the same dts
    Gc = oracle.grow(p.U0)
    Pc = oracle.params_of(p)
    for dt in dts:
        oracle.fill_domain(Gc, Pc)
        Gc, _ = oracle.advance_box(Gc, Pc, dt)
    err_fine = np.abs(Uf[0] - ref_patch[0]).max()
    coarse_on_fine = np.repeat(np.repeat(np.repeat(oracle.valid(Gc)[0], 2, 0), 2, 1), 2, 2)
    err_coarse = np.abs(coarse_on_fine[flo[2]:flo[2] + nf[2], flo[1]:flo[1] + nf[1], flo[0]:flo[0] + nf[0]]
                        - ref_patch[0]).max()
    assert err_fine < 0.2 * err_coarse, (err_fine, err_coarse)


def test_fine_ghosts_interpolate_in_time():
    # coarse states linear in space at t^n and t^{n+1}: the ghost values at
    # theta are the fine cell averages of the linear field interpolated in time
    rng = np.random.default_rng(9)
    lo = np.array([2, 4, 6])
    shape = (6, 6, 6)
    k, j, i = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    X = np.stack([i + lo[0] + 0.5, j + lo[1] + 0.5, k + lo[2] + 0.5])
    fields = []
    for _ in range(2):
        g = rng.uniform(-1, 1, (5, 3))
        c0 = rng.uniform(1, 2, 5)
        fields.append((c0, g, np.stack([c0[m] + g[m] @ X.reshape(3, -1) for m in range(5)]).reshape((5,) + shape)))
    fine = np.array([[2 * (lo[0] + a) + p, 2 * (lo[1] + b) + q, 2 * (lo[2] + c) + r]
                     for a in (1, 3) for b in (2, 4) for c in (1, 4) for p in (0, 1) for q in (0, 1) for r in (0, 1)])
    centre = (fine + 0.5) / 2.0
    for theta in (0.0, 0.5):
        got = oracle.fine_ghost_values(fields[0][2], fields[1][2], theta, lo, fine)
        want = np.stack([(1 - theta) * (fields[0][0][m] + fields[0][1][m] @ centre.T)
                         + theta * (fields[1][0][m] + fields[1][1][m] @ centre.T) for m in range(5)])
        np.testing.assert_allclose(got, want, rtol=0, atol=2e-13)


# ---------------------------------------------------------------- several patches

def _patches_problem(n=24, patches=(((8, 8, 8), (16, 16, 16)),), field=None, vel=(1.0, 0.5, 0.25)):
    """Two-level problem whose fine level is the given half-open coarse ranges."""
    x, y, z = W.cell_centres((n, n, n))
    f = field or (lambda x, y, z: 1.0 + 0.2 * np.sin(2 * np.pi * (x + y + z)))
    p = W.Problem("tlp", (n, n, n), 1.4, W.conserved(1.4, f(x, y, z), *vel, 1.0),
                  W.regular_boxes((n, n, n), (n // 2,) * 3))
    p.fine_patches, p.fine_boxes = W.refine_patches(patches, (n, n, n), (8, 8, 8),
                                                lambda x, y, z: W.conserved(1.4, f(x, y, z), *vel, 1.0))
    return p


def _composite_total(p, Uc, Ufs, m):
    """Composite integral of component m: uncovered coarse cells plus fine cells / 8."""
    cov = np.zeros(Uc.shape[1:], bool)
    fine = []
    for (flo, _), Uf in zip(p.fine_patches, Ufs):
        c = np.array(flo) // 2
        nc = np.array(Uf.shape[1:][::-1]) // 2
        cov[c[2]:c[2] + nc[2], c[1]:c[1] + nc[1], c[0]:c[0] + nc[0]] = True
        fine.append(Uf[m].ravel() / 8.0)
    return math.fsum(np.concatenate([Uc[m][~cov].ravel()] + fine))


def test_split_patches_equal_one_rectangle():
    """A patch cut into touching rectangles (fine ghosts from the neighbour
    patch, no register on the faces between them) gives bitwise the state of
    the one rectangle."""
    whole = _patches_problem(patches=[((8, 8, 8), (16, 16, 16))])
    Uc1, Uf1, d1, _ = oracle.run_two_level(whole, 4)
    for cuts in ([((8, 8, 8), (12, 16, 16)), ((12, 8, 8), (16, 16, 16))],
                 [((8, 8, 8), (12, 12, 16)), ((12, 8, 8), (16, 12, 16)),
                  ((8, 12, 8), (12, 16, 16)), ((12, 12, 8), (16, 16, 16))]):
        split = _patches_problem(patches=cuts)
        Uc2, Ufs, d2, _ = oracle.run_two_level(split, 4)
        assert np.array_equal(Uc1, Uc2) and np.array_equal(d1, d2)
        for (flo, _), Uf in zip(split.fine_patches, Ufs):
            o = np.array(flo) - np.array(whole.fine_patches[0][0])
            n = np.array(Uf.shape[1:][::-1])
            assert np.array_equal(Uf, Uf1[:, o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0]])


def test_separated_patches_uniform_state_bitwise():
    p = _patches_problem(n=32, patches=[((4, 6, 8), (12, 14, 16)), ((18, 10, 12), (26, 20, 22))],
                         field=lambda x, y, z: np.full_like(x, 0.7), vel=(0.4, -0.3, 0.2))
    Uc, Ufs, dts, cnt = oracle.run_two_level(p, 3)
    for m in range(5):
        assert np.all(Uc[m] == p.U0[m].flat[0])
        for Uf in Ufs:
            assert np.all(Uf[m] == p.U0[m].flat[0])
    assert not cnt.any()


@pytest.mark.parametrize("patches", [
    [((6, 8, 8), (12, 16, 16)), ((13, 8, 8), (19, 16, 16))],    # a gap of one coarse cell: refluxed from both sides
    [((6, 6, 8), (12, 12, 16)), ((12, 12, 8), (18, 18, 16))],   # diagonal neighbours: corner cells beside both
])
def test_patches_composite_conservation(patches):
    p = _patches_problem(patches=patches)
    t0 = [_composite_total(p, p.U0, [U for _, U in p.fine_patches], m) for m in range(5)]
    Uc, Ufs, dts, cnt = oracle.run_two_level(p, 5)
    scale = math.fsum(np.abs(p.U0[0]).ravel())
    for m in range(5):
        assert abs(_composite_total(p, Uc, Ufs, m) - t0[m]) <= 1e-13 * scale
    # covered coarse cells are the average of their children
    for (flo, _), Uf in zip(p.fine_patches, Ufs):
        c = np.array(flo) // 2
        nf = np.array(Uf.shape[1:][::-1])
        cov = Uc[:, c[2]:c[2] + nf[2] // 2, c[1]:c[1] + nf[1] // 2, c[0]:c[0] + nf[0] // 2]
        avg = Uf.reshape(5, nf[2] // 2, 2, nf[1] // 2, 2, nf[0] // 2, 2).mean(axis=(2, 4, 6))
        np.testing.assert_allclose(cov, avg, rtol=1e-14, atol=1e-15)
