"""Parity of the HIP path with the oracle for problems with passive species.

Species (mass fractions X_s, conserved rho X_s after rho E) are advected with
the flow: traced and limited like the other primitives, carried by the
contact family and by the HLLC star state (section 4: the GPU proxy advects
13 species with the hydrodynamics).  Tolerances as for the hydro fields:
discontinuous inputs per-field L1 relative <= 1e-8, totals <= 1e-13; the HIP path
aims at bitwise equality and the tests report the largest difference.
"""
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
def test_kh_three_species_ragged_boxes(ctx, form):
    prob = W.kelvin_helmholtz(n=(40, 36, 20), box=(16, 16, 20), nspec=3)
    assert prob.U0.shape[0] == 8
    ref, _, cref = oracle.run_problem(prob, 10)
    got, cnt = _run_gpu(ctx, prob, 10, form)
    _report(f"kh species {form}", got, ref)
    _check(got, ref)
    assert not cnt[:5].any() and not cref.any()


def test_rt_two_species_reflect_gravity(ctx):
    prob = W.rayleigh_taylor(n=(32, 16, 48), seed=11, nspec=2)
    ref, _, cref = oracle.run_problem(prob, 12)
    got, cnt = _run_gpu(ctx, prob, 12)
    _report("rt species", got, ref)
    _check(got, ref)
    assert not cnt[:5].any() and not cref.any()


def test_sixteen_species_smooth(ctx):
    prob = W.serving_request(seed=77, n=24, nspec=16)
    ref, _, _ = oracle.run_problem(prob, 8)
    got, cnt = _run_gpu(ctx, prob, 8)
    _report("16 species", got, ref)
    assert max(max_rel(got, ref)) <= 1e-10
    assert not cnt[:5].any()


def test_cloud_two_level_species_inflow(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.cloud_wind(n=32, box=16, fine_box=16, nspec=3)
    assert prob.inflow_X and len(prob.inflow_X) == 3
    rc, rf, _, _ = oracle.run_two_level(prob, 8)
    s = ctuppm.Solver(ctx, prob, form="batched")
    s.step(8)
    gc, gf = s.state(), s.state_fine()
    s.close()
    _report("cloud species coarse", gc, rc)
    _report("cloud species fine", gf, rf)
    _check(gc, rc)
    _check(gf, rf)


def test_mixed_species_batch_equals_alone(ctx):
    """Problems with different species counts share one batched launch set;
    each must equal its own run alone, bitwise."""
    from paper_1711_06203_amd import ctuppm
    probs = [W.serving_request(seed=300, n=16, nspec=0), W.serving_request(seed=301, n=24, nspec=13),
             W.kelvin_helmholtz(n=(24, 20, 16), box=(12, 20, 16), nspec=2)]
    alone = [_run_gpu(ctx, p, 5)[0] for p in probs]
    for form in ("batched", "graph"):
        solvers = [ctuppm.Solver(ctx, p, form=form) for p in probs]
        ctx.step(solvers, form, 5)
        for s, a in zip(solvers, alone):
            assert np.array_equal(s.state(), a)
            s.close()


def test_species_bad_count_rejected(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.serving_request(seed=5, n=8, nspec=2)
    prob.nspec = 17
    with pytest.raises((ctuppm.CtuError, ValueError)):
        ctuppm.Solver(ctx, prob)
