"""Checkpoint and resume on the GPU: a run stopped, saved, resumed in a new
solver and continued equals the uninterrupted run bitwise -- single level
with species, the method of lines with a fixed dt, and two levels after the
fine level moved."""
import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import regrid, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


@pytest.mark.parametrize("form", ["batched", "graph"])
def test_single_level_species(ctx, tmp_path, form):
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=(40, 36, 20), box=(16, 16, 20), nspec=2)
    p = str(tmp_path / "kh.npz")
    s = ctuppm.Solver(ctx, prob, form=form)
    s.step(3)
    s.checkpoint(p)
    s.step(3)
    a = s.state()
    s.close()
    r = ctuppm.Solver.resume(ctx, p, form=form)
    assert r.steps_before == 3
    r.step(3)
    b = r.state()
    r.checkpoint(str(tmp_path / "kh2.npz"))
    r.close()
    ref, _, _ = oracle.run_problem(prob, 6)
    assert np.array_equal(a, b) and np.array_equal(b, ref)
    from paper_1711_06203_amd import checkpoint
    _, meta = checkpoint.load(str(tmp_path / "kh2.npz"))
    assert meta["steps_taken"] == 6


def test_method_of_lines_fixed_dt(ctx, tmp_path):
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=32, box=16, nspec=1)
    prob.scheme = 2
    p = str(tmp_path / "mol.npz")
    s = ctuppm.Solver(ctx, prob, fixed_dt=2e-3)
    s.step(2)
    s.checkpoint(p)
    s.step(2)
    a = s.state()
    s.close()
    r = ctuppm.Solver.resume(ctx, p)
    assert r.fixed_dt == 2e-3
    r.step(2)
    b = r.state()
    r.close()
    ref, _, _ = oracle.run_problem(prob, 4, dt_fixed=2e-3)
    assert np.array_equal(a, b) and np.array_equal(b, ref)


def test_two_levels_after_a_regrid(ctx, tmp_path):
    from paper_1711_06203_amd import ctuppm
    prob = W.cloud_wind(n=32, box=16, fine_box=16, fine_region=((8, 8, 8), (24, 24, 24)), nspec=1)
    p = str(tmp_path / "cloud.npz")
    s = ctuppm.Solver(ctx, prob)
    s.step(2)
    s.regrid(regrid.fine_boxes(((10, 8, 8), (25, 23, 23)), fine_box=16))
    s.step(1)
    s.checkpoint(p)
    s.step(2)
    ac, af = s.state(), s.state_fine()
    s.close()
    r = ctuppm.Solver.resume(ctx, p)
    assert r.fine_lo == (20, 16, 16)
    r.step(2)
    bc, bf = r.state(), r.state_fine()
    r.close()
    assert np.array_equal(ac, bc) and np.array_equal(af, bf)
