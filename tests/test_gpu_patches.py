"""A fine level made of several patches (section 3, figure 1: fine boxes over
separate parts of the coarse level), on the GPU against the oracle.

The fine boxes of different patches exchange ghost cells with each other,
the coarse level fills the rest, the flux register holds only the faces
between a patch and an uncovered coarse cell, and a coarse cell beside the
fine level on several sides (in a one-cell gap, at a corner between
diagonal patches) is refluxed in a fixed order of face groups.  Every case is
bitwise the oracle's, patch by patch."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


def _smooth(n, patches, fine_edge=(8, 8, 8)):
    f = lambda x, y, z: 1.0 + 0.2 * np.sin(2 * np.pi * (x + y + z))
    state = lambda x, y, z: W.conserved(1.4, f(x, y, z), 1.0, 0.5, 0.25, 1.0)
    p = W.Problem("tlp", (n, n, n), 1.4, state(*W.cell_centres((n, n, n))), W.regular_boxes((n, n, n), (n // 2,) * 3))
    p.fine_patches, p.fine_boxes = W.refine_patches(patches, (n, n, n), fine_edge, state)
    return p


def _oracle(prob, steps):
    rc, rf, dts, cnt = oracle.run_two_level(prob, steps)
    return rc, ([rf] if isinstance(rf, np.ndarray) else rf), dts, cnt


def _gpu(ctx, prob, steps, form):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form=form)
    s.step(steps)
    out = s.state(), s.state_patches(), s.dt(), s.counters()
    s.close()
    return out


def _equal(name, got, want):
    gc, gfs = got[0], got[1]
    rc, rfs = want[0], want[1]
    ok = [np.array_equal(gc, rc)] + [np.array_equal(g, r) for g, r in zip(gfs, rfs)]
    print(f"{name}: coarse and patches bitwise {ok}", flush=True)
    assert len(gfs) == len(rfs) and all(ok)


@pytest.mark.parametrize("form", ["batched", "graph"])
@pytest.mark.parametrize("patches", [
    [((6, 8, 8), (12, 16, 16)), ((13, 8, 8), (19, 16, 16))],        # a one-cell coarse gap
    [((6, 6, 8), (12, 12, 16)), ((12, 12, 8), (18, 18, 16))],       # diagonal neighbours
    [((8, 8, 8), (12, 12, 16)), ((12, 8, 8), (16, 12, 16)),          # one rectangle in four patches
     ((8, 12, 8), (12, 16, 16)), ((12, 12, 8), (16, 16, 16))],
])
def test_patch_layouts_equal_the_oracle(ctx, form, patches):
    prob = _smooth(24, patches)
    want = _oracle(prob, 4)
    got = _gpu(ctx, prob, 4, form)
    _equal(f"{len(patches)} patches {form}", got, want)
    assert got[2] == want[2][-1]


def test_two_clouds_twenty_coarse_steps(ctx):
    """Two dense clouds in a Mach-2 wind, each refined by its own patch."""
    prob = W.two_clouds(n=64, box=16, fine_box=16)
    assert len(prob.fine_patches) == 2
    want = _oracle(prob, 20)
    got = _gpu(ctx, prob, 20, "graph")
    _equal("two clouds 64^3, 20 coarse steps", got, want)
    assert not got[3][:5].any() and not want[3].any()


def test_two_clouds_in_pieces_equal_one_call(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.two_clouds(n=48, box=16, fine_box=8, nspec=2)
    a = ctuppm.Solver(ctx, prob)
    a.step(3)
    ga = (a.state(), a.state_patches())
    a.close()
    b = ctuppm.Solver(ctx, prob)
    b.step_in_pieces(3)
    gb = (b.state(), b.state_patches())
    b.close()
    assert np.array_equal(ga[0], gb[0]) and all(np.array_equal(x, y) for x, y in zip(ga[1], gb[1]))
    want = _oracle(prob, 3)
    _equal("two clouds 48^3 with 2 species", ga, want)


def test_patches_of_uneven_boxes(ctx):
    """Patches tiled by boxes of several sizes (a ragged tail per patch)."""
    prob = _smooth(32, [((5, 6, 7), (14, 15, 13)), ((17, 6, 7), (26, 18, 19))], fine_edge=(8, 6, 10))
    sizes = {tuple(b[1][d] - b[0][d] + 1 for d in range(3)) for b in prob.fine_boxes}
    assert len(sizes) > 1
    want = _oracle(prob, 3)
    got = _gpu(ctx, prob, 3, "batched")
    _equal("uneven boxes in two patches", got, want)


def test_regrid_onto_two_patches(ctx):
    """One rectangle moved onto two patches (cells under the old one copied,
    the rest interpolated), then stepped."""
    from paper_1711_06203_amd import ctuppm, regrid
    prob = W.cloud_wind(n=32, box=16, fine_box=8, fine_region=((10, 10, 10), (22, 22, 22)))
    s = ctuppm.Solver(ctx, prob)
    s.step(2)
    rc, rf, _, _ = oracle.run_two_level(prob, 2)
    new = [((8, 9, 10), (15, 20, 21)), ((18, 9, 10), (25, 16, 17))]
    boxes, rects = regrid.fine_level(new, fine_box=8)
    s.regrid(boxes, rects)
    want = oracle.regrid_patches(rc, [(prob.fine_lo, rf)], rects)
    for g, w in zip(s.state_patches(), want):
        assert np.array_equal(g, w)
    s.step(2)
    p2 = dataclasses.replace(prob, U0=rc, fine_patches=[(lo, U) for (lo, _), U in zip(rects, want)],
                             U0_fine=None, fine_lo=None)
    want2 = _oracle(p2, 2)
    _equal("after regrid onto two patches", (s.state(), s.state_patches()), want2)
    s.close()
