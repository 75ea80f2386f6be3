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


def test_adapt_follows_the_tags(ctx):
    """Tag -> cluster -> regrid in a loop; the oracle takes the same patches
    (computed from its own tags) and the states agree."""
    from paper_1711_06203_amd import ctuppm, regrid
    prob = W.cloud_wind(n=32, box=16, fine_box=16, fine_region=((12, 12, 12), (20, 20, 20)))
    s = ctuppm.Solver(ctx, prob)
    Uc, Uf, flo = prob.U0, prob.U0_fine, prob.fine_lo
    moved = 0
    for cycle in range(3):
        s.step(2)
        Uc, Uf, _, _ = oracle.run_two_level_from(prob, Uc, Uf, flo, 2)
        patch_o = regrid.patch_from_tags(oracle.tag_cells(Uc, oracle.params_of(prob), 0.05), buffer=2)
        boxes = regrid.adapt(s, 0.05, buffer=2, fine_box=16)
        cur = (tuple(v // 2 for v in flo), tuple((flo[d] + Uf.shape[3 - d]) // 2 - 1 for d in range(3)))
        if patch_o is not None and patch_o != cur:
            assert boxes is not None
            new_lo = tuple(2 * v for v in patch_o[0])
            new_n = tuple(2 * (patch_o[1][d] - patch_o[0][d] + 1) for d in range(3))
            Uf = oracle.regrid_fine(Uc, Uf, flo, new_lo, new_n)
            flo = new_lo
            moved += 1
        else:
            assert boxes is None
        _check(s.state(), Uc)
        _check(s.state_fine(), Uf)
    assert moved >= 1
    s.close()
