"""Parity of the HIP path with the oracle for CW84 contact steepening (CTU and
MOL, one and two levels).  Tolerances as elsewhere; bitwise equality is
reported."""
import numpy as np
import pytest

import oracle
from gpu_helpers import l1_rel, max_rel, totals_rel
from paper_1711_06203_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


def _run_gpu(ctx, prob, nsteps, form="batched"):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form=form)
    s.step(nsteps)
    out = s.state()
    cnt = s.counters()
    s.close()
    return out, cnt


def _report(name, got, ref):
    d = np.abs(got - ref)
    print(f"{name}: bitwise={np.array_equal(got, ref)} max_abs={d.max():.3e} "
          f"max_rel={max(max_rel(got, ref)):.3e} l1={max(l1_rel(got, ref)):.3e}", flush=True)


def _check(got, ref):
    assert got.shape == ref.shape
    assert max(l1_rel(got, ref)) <= 1e-8
    assert max(totals_rel(got, ref)) <= 1e-13


@pytest.mark.parametrize("form", ["per_box", "batched", "graph"])
def test_steepened_sod(ctx, form):
    prob = W.sod(n=32, steps=20)
    prob.steepen = 1
    ref, _, _ = oracle.run_problem(prob)
    got, cnt = _run_gpu(ctx, prob, 20, form)
    _report(f"steepen sod32 {form}", got, ref)
    _check(got, ref)
    assert not cnt[:5].any()


@pytest.mark.parametrize("scheme", [0, 1])
def test_steepened_kh_species_ragged(ctx, scheme):
    prob = W.kelvin_helmholtz(n=(40, 36, 20), box=(16, 16, 20), nspec=2)
    prob.steepen = 1
    prob.scheme = scheme
    ref, _, _ = oracle.run_problem(prob, 10)
    got, cnt = _run_gpu(ctx, prob, 10, "graph")
    _report(f"steepen kh scheme{scheme}", got, ref)
    _check(got, ref)


def test_steepened_contact_advection(ctx):
    N = 64
    nn = (N, 8, 8)
    x, y, z = W.cell_centres(nn)
    rho = np.where(np.abs(x - 0.3) < 0.15, 1.0, 0.125)
    U0 = W.conserved(1.4, rho, 1.0, 0.2, 0.0, 1.0)
    prob = W.Problem("contact", nn, 1.4, U0, W.regular_boxes(nn, (16, 8, 8)), steepen=1)
    ref, _, _ = oracle.run_problem(prob, 60)
    got, _ = _run_gpu(ctx, prob, 60)
    _report("steepen contact", got, ref)
    _check(got, ref)


def test_steepened_two_level_cloud_with_two_shock(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.cloud_wind(n=32, box=16, fine_box=16)
    prob.steepen = 1
    prob.riemann = 1
    rc, rf, _, _ = oracle.run_two_level(prob, 6)
    s = ctuppm.Solver(ctx, prob)
    s.step(6)
    gc, gf = s.state(), s.state_fine()
    s.close()
    _report("steepen cloud coarse", gc, rc)
    _report("steepen cloud fine", gf, rf)
    _check(gc, rc)
    _check(gf, rf)


def test_steepening_requires_the_cw84_limiter(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.sod(n=16)
    prob.steepen = 1
    prob.limiter = 1
    with pytest.raises(ctuppm.CtuError):
        ctuppm.Solver(ctx, prob)
