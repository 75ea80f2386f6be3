"""Dynamic regridding on the GPU against the oracle: the density-jump tags,
the new fine state of a regrid (copy from the old patch, conservative
interpolation from the coarse level), and stepping on after a regrid, all
through the C ABI.  Tags are integers: compared exactly; states: the usual
tolerances, with bitwise equality reported."""
import numpy as np
import pytest

import oracle
from gpu_helpers import l1_rel, totals_rel
from paper_1711_06203_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


def _report(name, got, ref):
    print(f"{name}: bitwise={np.array_equal(got, ref)} max_abs={np.abs(got - ref).max():.3e}", flush=True)


def _check(got, ref):
    assert got.shape == ref.shape
    assert max(l1_rel(got, ref)) <= 1e-8
    assert max(totals_rel(got, ref)) <= 1e-13


def test_tags_equal_the_oracle(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=(32, 40, 24), box=(16, 20, 24), nspec=1)
    s = ctuppm.Solver(ctx, prob)
    s.step(3)
    got_state = s.state()
    ref, _, _ = oracle.run_problem(prob, 3)  # the oracle's own state after three steps
    _check(got_state, ref)
    for thr in (0.01, 0.05, 0.2):
        tg = s.tag(thr)
        to = oracle.tag_cells(ref, oracle.params_of(prob), thr)
        assert np.array_equal(tg, to), thr
        assert tg.any()
    assert np.array_equal(s.state(), got_state)  # tagging leaves the valid cells alone
    s.close()


def test_regrid_then_step_equals_the_oracle(ctx):
    from paper_1711_06203_amd import ctuppm, regrid
    prob = W.cloud_wind(n=32, box=16, fine_box=16, nspec=1)
    s = ctuppm.Solver(ctx, prob)
    s.step(3)
    rc, rf, _, _ = oracle.run_two_level(prob, 3)
    gc, gf = s.state(), s.state_fine()
    _check(gc, rc)
    _check(gf, rf)
    # move the patch: coarse cells (10, 7, 8)..(25, 22, 23), fine boxes of 16
    patch = ((10, 7, 8), (25, 22, 23))
    boxes = regrid.fine_boxes(patch, 16)
    s.regrid(boxes)
    new_lo = tuple(2 * v for v in patch[0])
    new_n = tuple(2 * (patch[1][d] - patch[0][d] + 1) for d in range(3))
    want = oracle.regrid_fine(rc, rf, prob.fine_lo, new_lo, new_n)
    got = s.state_fine()
    _report("regrid fine state", got, want)
    _check(got, want)
    assert np.array_equal(s.state(), gc)  # the coarse level is untouched
    s.step(3)
    rc2, rf2, _, _ = oracle.run_two_level_from(prob, rc, want, new_lo, 3)
    gc2, gf2 = s.state(), s.state_fine()
    _report("after regrid coarse", gc2, rc2)
    _report("after regrid fine", gf2, rf2)
    _check(gc2, rc2)
    _check(gf2, rf2)
    s.close()


def _oracle_patches(prob, Uc, patches, nsteps):
    """The oracle's two-level run from a coarse state and fine patches [(lo, U)]."""
    import dataclasses
    p2 = dataclasses.replace(prob, U0=Uc, fine_patches=patches, U0_fine=None, fine_lo=None)
    Uc2, Ufs, _, _ = oracle.run_two_level(p2, nsteps)
    Ufs = [Ufs] if isinstance(Ufs, np.ndarray) else Ufs
    return Uc2, [(lo, U) for (lo, _), U in zip(patches, Ufs)]


def test_adapt_follows_the_tags(ctx):
    """Tag -> cluster -> regrid in a loop, every cluster a fine patch of its
    own; the oracle takes the same patches (computed from its own tags) and
    the states agree, patch by patch."""
    from paper_1711_06203_amd import ctuppm, regrid
    prob = W.two_clouds(n=48, box=16, fine_box=8)
    s = ctuppm.Solver(ctx, prob)
    Uc, pats = prob.U0, [(tuple(lo), U) for lo, U in prob.fine_patches]
    moved = 0
    for cycle in range(3):
        s.step(2)
        Uc, pats = _oracle_patches(prob, Uc, pats, 2)
        new_o = regrid.patches_from_tags(oracle.tag_cells(Uc, oracle.params_of(prob), 0.05), buffer=2)
        got = regrid.adapt(s, 0.05, buffer=2, fine_box=8)
        cur = [(tuple(lo[d] // 2 for d in range(3)), tuple((lo[d] + U.shape[3 - d]) // 2 - 1 for d in range(3)))
               for lo, U in pats]
        if new_o and sorted(new_o) != sorted(cur):
            assert got is not None and sorted(got) == sorted(new_o)
            rects = [(tuple(2 * c for c in lo), tuple(2 * (hi[d] - lo[d] + 1) for d in range(3))) for lo, hi in got]
            Ufs = oracle.regrid_patches(Uc, pats, rects)
            pats = [(lo, U) for (lo, _), U in zip(rects, Ufs)]
            moved += 1
        else:
            assert got is None
        _check(s.state(), Uc)
        for g, (lo, U) in zip(s.state_patches(), pats):
            _check(g, U)
    assert moved >= 1 and len(pats) >= 2
    s.close()
