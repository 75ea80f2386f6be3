"""Serving (continuous batching under an HBM budget) and autotuning on the GPU.

Each served result must equal the same problem advanced alone (bitwise: a
problem's arithmetic does not depend on what it is batched with), and the
alone result must match the CPU oracle; admission must respect the budget;
tuning choices must not change results.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import max_rel
from paper_1711_06203_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


def _alone(ctx, prob, steps):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form="batched")
    s.step(steps)
    out = s.state()
    s.close()
    return out


def test_served_results_equal_alone_and_oracle(ctx):
    from paper_1711_06203_amd import serving
    sizes = (16, 24, 32, 20)
    reqs = []
    for r in range(7):
        prob = W.serving_request(seed=1000 + r, n=sizes[r % len(sizes)], steps=6 + r % 3)
        reqs.append(serving.Request(r, prob, 0.0, prob.steps))
    # at most three resident at a time: later requests are admitted as slots free up
    srv = serving.Server(ctx, hbm_budget=1e12, keep_states=True, max_active=3)
    res = srv.run(reqs, realtime=False)
    assert len(res) == len(reqs)
    assert max(srv.batch_sizes) == 3 and min(srv.batch_sizes) >= 1
    for req in reqs:
        got = res[req.rid].state
        alone = _alone(ctx, req.prob, req.steps)
        assert np.array_equal(got, alone), req.rid
    ref, _, _ = oracle.run_problem(reqs[0].prob, reqs[0].steps)
    assert max(max_rel(res[0].state, ref)) <= 1e-10


def test_a_rejected_step_is_redone_and_reported(ctx):
    """A served problem whose update fails once (host-set hook) is not
    committed there: the rejection is reported with its result, the step is
    taken again, and the result still equals the problem advanced alone."""
    from paper_1711_06203_amd import serving
    reqs = []
    for r in range(4):
        prob = W.serving_request(seed=3000 + r, n=(16, 24)[r % 2], steps=8)
        reqs.append(serving.Request(r, prob, 0.0, 8, fail_step=3 if r == 1 else None))
    srv = serving.Server(ctx, hbm_budget=1e12, keep_states=True)
    res = srv.run(reqs, realtime=False)
    assert res[1].rejected >= 1 and not res[1].failed
    assert all(res[r].rejected == 0 for r in (0, 2, 3))
    for req in reqs:
        assert res[req.rid].steps == 8
        assert np.array_equal(res[req.rid].state, _alone(ctx, req.prob, 8)), req.rid


def test_admission_overlaps_steps_in_flight(ctx):
    """Admitting a problem while others are stepping enqueues its upload on a
    side stream: the served results are unchanged."""
    from paper_1711_06203_amd import serving
    reqs = [serving.Request(r, W.serving_request(seed=4000 + r, n=(32, 16)[r % 2], steps=5), 0.002 * r, 5)
            for r in range(6)]
    srv = serving.Server(ctx, hbm_budget=1e12, keep_states=True)
    res = srv.run(reqs, realtime=True)
    for req in reqs:
        assert np.array_equal(res[req.rid].state, _alone(ctx, req.prob, 5)), req.rid


def test_admission_respects_hbm_budget(ctx):
    from paper_1711_06203_amd import serving
    reqs = [serving.Request(r, W.serving_request(seed=2000 + r, n=24, steps=3), 0.0, 3) for r in range(5)]
    need = serving.footprint_bytes(reqs[0].prob)
    srv = serving.Server(ctx, hbm_budget=2.5 * need, keep_states=False)
    res = srv.run(reqs, realtime=False)
    assert len(res) == 5
    assert max(srv.batch_sizes) == 2
    assert srv.used == 0


def test_poisson_stream_latency_stats(ctx):
    from paper_1711_06203_amd import serving
    reqs = serving.poisson_requests(6, rate=200.0, seed=5, steps=4, sizes=(16, 24))
    srv = serving.Server(ctx, hbm_budget=1e12)
    res = srv.run(reqs, realtime=True)
    st = serving.latency_stats(res)
    assert st["count"] == 6 and 0 < st["p50_s"] <= st["p99_s"]


def test_tuning_does_not_change_results(ctx):
    from paper_1711_06203_amd import autotune, ctuppm
    prob = W.rayleigh_taylor(n=48, seed=8, boxes=W.uneven_boxes((48, 48, 48), 8, edges=(16, 32)))
    outs = []
    for bpc, zseg, ytile in ((0, 1, 0), (16, 4, 3), (4, 3, 8)):
        ctx.set_tuning(bpc, zseg, 2, ytile)
        s = ctuppm.Solver(ctx, prob, form="graph")
        s.step(3)
        outs.append(s.state())
        s.close()
    ctx.set_tuning(0, 1, 1)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    s = ctuppm.Solver(ctx, prob, form="batched")
    best = autotune.tune(ctx, [s], candidates=((0, 1, 0), (8, 2, 4)), steps=1, cache=None)
    assert best["blocks_per_cu"] in (0, 8) and best["ms_per_step"] > 0
    s.close()
    ctx.set_tuning(0, 1, 1)
