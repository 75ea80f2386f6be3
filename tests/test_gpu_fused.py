"""The merged kernels (CTU: flattening and tracing of x, y, z in one kernel,
the first transverse stage of x, y, z in one kernel; method of lines:
flattening and the face states of x, y, z in one kernel; the species in a
stage of their own, or inside the merged kernels) against the
one-kernel-per-direction form: bitwise the same states for every scheme
variant, boundary kind, box layout and the two-level step, and all equal
the oracle."""
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
    c.set_fused(True)
    c.close()


def _kh(**kw):
    p = W.kelvin_helmholtz(n=(40, 36, 20), box=(16, 16, 20), nspec=2)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


CASES = {
    "kh_species": lambda: _kh(),
    "kh_cs_twoshock": lambda: _kh(limiter=1, riemann=1),
    "kh_steepen": lambda: _kh(steepen=1),
    "rt_walls_gravity": lambda: W.rayleigh_taylor(n=48, seed=5, boxes=W.uneven_boxes((48, 48, 48), 5, edges=(16, 32))),
    "sod_outflow": lambda: W.sod(n=(24, 16, 16), steps=4, boxes_edge=(8, 8, 16)),
    "cloud_two_level": lambda: W.cloud_wind(n=32, box=16, fine_box=8, fine_region=((10, 10, 10), (22, 22, 22)), nspec=1),
    "mol2_species": lambda: _kh(scheme=1),
    "mol3_cs_twoshock": lambda: _kh(scheme=2, limiter=1, riemann=1),
    "mol2_steepen": lambda: _kh(scheme=1, steepen=1),
}


def _run(ctx, prob, steps, form):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form=form)
    s.step(steps)
    out = [s.state()] + (s.state_patches() if prob.fine_boxes else []) + [s.counters()]
    s.close()
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_fused_equals_split_and_oracle(ctx, name):
    prob = CASES[name]()
    res = {}
    for fused in (1, 2, 0):
        ctx.set_fused(fused)
        for form in (["batched", "graph"] if prob.fine_boxes else ["per_box", "batched", "graph"]):
            res[(fused, form)] = _run(ctx, prob, 3, form)
    ctx.set_fused(True)
    ref = res[(1, "batched")]
    for key, got in res.items():
        assert all(np.array_equal(a, b) for a, b in zip(got, ref)), key
    if prob.fine_boxes:
        rc, rf, _, _ = oracle.run_two_level(prob, 3)
        assert np.array_equal(ref[0], rc) and np.array_equal(ref[1], rf)
    else:
        U, _, _ = oracle.run_problem(prob, 3)
        assert np.array_equal(ref[0], U)


def test_fused_mode_refused(ctx):
    from paper_1711_06203_amd import ctuppm
    for bad in (3, -1):
        with pytest.raises((ctuppm.CtuError, ValueError)):
            ctx.set_fused(bad)
    with pytest.raises(ctuppm.CtuError):
        ctx.call("ctuppm_set_fused", 3)
    ctx.set_fused(True)
