"""Uninitialised reads: before every step the whole workspace after the
library's device tables (stage scratch, Runge-Kutta stage fabs, two-level
buffers and flux register) is set to NaN bytes, the fab the step writes is set to NaN and so are the ghost cells of
the current one.  A kernel that read a value the step had not written would
carry a NaN (or a different value) into the result; every case must still
equal the oracle bitwise."""
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


def _poison(s):
    nan = float("nan")
    s.ws[s.meta_bytes():].fill_(255)  # every byte 0xff: every double a NaN
    for lev, L in enumerate(s.lv):
        which = s.current() if lev == 0 else 0  # the fine level is back in its A fabs after a step
        cur, other = (L["A"], L["B"]) if which == 0 else (L["B"], L["A"])
        other.fill_(nan)
        for o, shp in zip(L["offsets"], L["shapes"]):
            v = cur[o:o + int(np.prod(shp))].view(shp)
            inner = v[:, 4:-4, 4:-4, 4:-4].clone()
            v.fill_(nan)
            v[:, 4:-4, 4:-4, 4:-4] = inner


def _run_poisoned(ctx, prob, nsteps, form):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form=form)
    for _ in range(nsteps):
        _poison(s)
        s.step(1)
    out = (s.state(), s.state_fine() if prob.fine_boxes else None)
    s.close()
    return out


def _kh_ragged(**kw):
    prob = W.kelvin_helmholtz(n=(40, 36, 20), box=(16, 16, 20), nspec=2)
    for k, v in kw.items():
        setattr(prob, k, v)
    return prob


@pytest.mark.parametrize("form", ["per_box", "batched", "graph"])
def test_ctu_ragged_boxes_species(ctx, form):
    prob = _kh_ragged()
    got, _ = _run_poisoned(ctx, prob, 4, form)
    ref, _, _ = oracle.run_problem(prob, 4)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("variant", [dict(scheme=2), dict(scheme=1, riemann=1, limiter=1), dict(steepen=1),
                                     dict(riemann=1)])
def test_variants(ctx, variant):
    prob = _kh_ragged(**variant)
    got, _ = _run_poisoned(ctx, prob, 3, "graph")
    ref, _, _ = oracle.run_problem(prob, 3)
    assert np.array_equal(got, ref), variant


def test_walls_gravity_uneven_boxes(ctx):
    prob = W.rayleigh_taylor(n=(32, 16, 48), seed=11, nspec=1)
    got, _ = _run_poisoned(ctx, prob, 4, "batched")
    ref, _, _ = oracle.run_problem(prob, 4)
    assert np.array_equal(got, ref)


def test_outflow_one_box_per_box_form(ctx):
    prob = W.sod(n=(32, 8, 8), boxes_edge=(32, 8, 8))
    got, _ = _run_poisoned(ctx, prob, 5, "per_box")
    ref, _, _ = oracle.run_problem(prob, 5)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("form", ["batched", "graph"])
def test_two_level_inflow_species(ctx, form):
    prob = W.cloud_wind(n=32, box=16, fine_box=16, fine_region=((8, 8, 8), (24, 24, 24)), nspec=1)
    gc, gf = _run_poisoned(ctx, prob, 3, form)
    rc, rf, _, _ = oracle.run_two_level(prob, 3)
    assert np.array_equal(gc, rc) and np.array_equal(gf, rf)


def test_the_poison_reaches_the_result_when_a_read_value_is_poisoned(ctx):
    """Control: poisoning valid cells of the current state (values the step
    does read) shows up as NaNs in the result and in the failure counter, so
    a clean result above means no poisoned value was read."""
    from paper_1711_06203_amd import ctuppm
    prob = _kh_ragged()
    s = ctuppm.Solver(ctx, prob, form="batched")
    _poison(s)
    L = s.lv[0]
    o, shp = L["offsets"][0], L["shapes"][0]
    v = L["A"][o:o + int(np.prod(shp))].view(shp)
    v[0, 8, 8, 8] = float("nan")
    s.step(1)
    got, cnt = s.state(), s.counters()
    s.close()
    assert np.isnan(got).any() and cnt[4] > 0
