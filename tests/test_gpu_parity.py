"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: smooth inputs after 10 steps, per-field max|g-o|/max|o| <= 1e-10;
inputs with shocks or contacts, per-field L1 relative <= 1e-8; conserved
totals <= 1e-13 relative; floor and failure counters equal (zero).  The HIP path
aims at bitwise equality (no contraction on either side); the tests report
the largest difference seen.
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


def _run_gpu(ctx, prob, nsteps, form="batched", fixed_dt=None):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form=form, fixed_dt=fixed_dt)
    s.step(nsteps)
    out = s.state()
    cnt = s.counters()
    dt = s.dt()
    s.close()
    return out, cnt, dt


def _report(name, got, ref):
    d = np.abs(got - ref)
    print(f"{name}: bitwise={np.array_equal(got, ref)} max_abs={d.max():.3e} "
          f"max_rel={max(max_rel(got, ref)):.3e} l1={max(l1_rel(got, ref)):.3e}", flush=True)


@pytest.mark.parametrize("form", ["per_box", "batched", "graph"])
def test_sod_32_single_box(ctx, form):
    prob = W.sod(n=32, steps=20)
    ref, dts, cref = oracle.run_problem(prob)
    got, cnt, dt = _run_gpu(ctx, prob, 20, form)
    _report(f"sod32 {form}", got, ref)
    assert max(l1_rel(got, ref)) <= 1e-8
    assert max(totals_rel(got, ref)) <= 1e-13
    assert dt == pytest.approx(dts[-1], rel=1e-13)
    assert not cnt[:5].any() and not cref.any()
    assert cnt[5] == 20


def test_box_decomposition_is_bitwise_invisible(ctx):
    one = W.sod(n=(32, 24, 16), steps=6)
    many = W.sod(n=(32, 24, 16), steps=6, boxes_edge=(8, 8, 8))
    a, _, _ = _run_gpu(ctx, one, 6)
    b, _, _ = _run_gpu(ctx, many, 6)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n,edge", [((13, 7, 9), None), ((40, 24, 20), (16, 8, 20)), ((24, 40, 17), (24, 8, 17))])
def test_ragged_boxes_smooth(ctx, n, edge):
    prob = W.serving_request(seed=7, n=8)
    # a smooth periodic state on an odd-shaped domain
    x, y, z = W.cell_centres(n)
    rho = 1.0 + 0.1 * np.sin(2 * np.pi * (x + 2 * y)) * np.cos(2 * np.pi * z)
    U = W.conserved(1.4, rho, 0.3 * np.sin(2 * np.pi * y), 0.2 * np.cos(2 * np.pi * x), 0.1,
                    1.0 + 0.1 * np.cos(2 * np.pi * (x - z)))
    boxes = W.regular_boxes(n, edge or n)
    prob = W.Problem("ragged", n, 1.4, U, boxes, cfl=0.5)
    ref, _, _ = oracle.run_problem(prob, 10)
    got, cnt, _ = _run_gpu(ctx, prob, 10)
    _report(f"ragged {n}", got, ref)
    assert max(max_rel(got, ref)) <= 1e-10
    assert not cnt[:5].any()


def test_smooth_serving_ic_32(ctx):
    prob = W.serving_request(seed=123, n=32)
    ref, _, _ = oracle.run_problem(prob, 10)
    got, cnt, _ = _run_gpu(ctx, prob, 10)
    _report("serving32", got, ref)
    assert max(max_rel(got, ref)) <= 1e-10
    assert max(totals_rel(got, ref)) <= 1e-13


def test_kelvin_helmholtz_small(ctx):
    prob = W.kelvin_helmholtz(n=48, box=24, seed=9)
    ref, _, _ = oracle.run_problem(prob, 10)
    got, cnt, _ = _run_gpu(ctx, prob, 10)
    _report("kh48", got, ref)
    assert max(l1_rel(got, ref)) <= 1e-8
    assert max(totals_rel(got, ref)) <= 1e-13


def test_rayleigh_taylor_uneven_boxes(ctx):
    prob = W.rayleigh_taylor(n=96, seed=3)
    assert len(prob.boxes) > 8
    ref, _, cref = oracle.run_problem(prob, 5)
    got, cnt, _ = _run_gpu(ctx, prob, 5)
    _report("rt96", got, ref)
    assert max(l1_rel(got, ref)) <= 1e-8
    assert not cnt[:5].any() and not cref.any()


def test_uniform_state_stays_bitwise_uniform(ctx):
    prob = W.uniform(n=(24, 16, 16), box=8)
    got, cnt, _ = _run_gpu(ctx, prob, 4)
    for m in range(5):
        assert np.all(got[m] == prob.U0[m][0, 0, 0])


def test_forms_bitwise_equal(ctx):
    prob = W.rayleigh_taylor(n=48, seed=5, boxes=W.uneven_boxes((48, 48, 48), 5, edges=(16, 32)))
    res = [_run_gpu(ctx, prob, 3, f)[0] for f in ("per_box", "batched", "graph")]
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[1], res[2])


def test_retry_equals_explicit_half_steps(ctx):
    # a failure forced at step 2 (host hook) makes the checked step redo it as
    # two half steps; the result must equal running those half steps directly
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=24, box=12, seed=3)
    a = ctuppm.Solver(ctx, prob, form="batched")
    a.set_fail_hook(2)
    flags = [a.step_checked() for _ in range(4)]
    assert flags == [0, 0, 1, 0]  # halvings used: only step 2 was redone, as two halves
    got = a.state()
    a.close()
    b = ctuppm.Solver(ctx, prob, form="batched")
    b.step(2)
    # dt of step 2: the oracle's CFL rule on its own state after two steps
    P = oracle.params_of(prob)
    U2, _, _ = oracle.run(prob.U0, P, 2)
    G = oracle.fill_domain(oracle.grow(U2), P)
    dt2 = P.cfl / oracle.signal_speed(G, P)
    ctx.call("ctuppm_set_fixed_dt", b.pid, 0.5 * dt2)
    b.step(2)
    ctx.call("ctuppm_set_fixed_dt", b.pid, 0.0)
    b.step(1)
    want = b.state()
    b.close()
    assert np.array_equal(got, want)


def test_concurrent_graph_equals_serial_graph(ctx):
    """The graph form with the three directions on three streams gives the
    same bits as the single-chain graph and as the batched form."""
    from paper_1711_06203_amd import ctuppm
    probs = [W.kelvin_helmholtz(n=(40, 36, 20), box=(16, 16, 20), nspec=1), W.serving_request(seed=31, n=24)]
    out = {}
    for mode in ("serial", "concurrent", "batched"):
        ctx.set_concurrency(mode == "concurrent")
        solvers = [ctuppm.Solver(ctx, p) for p in probs]
        ctx.step(solvers, "batched" if mode == "batched" else "graph", 6)
        out[mode] = [s.state() for s in solvers]
        for s in solvers:
            s.close()
    ctx.set_concurrency(False)
    for a, b, c in zip(out["serial"], out["concurrent"], out["batched"]):
        assert np.array_equal(a, b) and np.array_equal(a, c)
