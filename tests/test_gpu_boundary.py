"""The C ABI's ownership and retry rules, through the binding.

* The library allocates no device memory: creating, stepping (every form),
  regridding and destroying many problems leaves the device memory outside
  PyTorch's allocator unchanged.
* Guarded steps: a step whose new state fails is not committed (U^n stays
  current, bitwise), the rejection reaches the host without a sync, and the
  next guarded call reports it (CTUPPM_ERETRY) until it is acknowledged.
* The checked step gives up with an accepted state current when even an
  eighth of the step fails.
* Stage dumps outside the bound workspace, or in a form a two-level problem
  does not step in, are refused before any copy.
* Re-binding the fine level does not change which fab holds the coarse state.
"""
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


def _outside_torch(torch):
    torch.cuda.synchronize()
    free, total = torch.cuda.mem_get_info()
    return total - free - torch.cuda.memory_reserved()


def _cycle(ctx, k):
    """Create, step in every form, regrid and destroy a few problems."""
    from paper_1711_06203_amd import ctuppm
    probs = [W.kelvin_helmholtz(n=(24, 16, 16), box=(8, 8, 16), seed=k, nspec=k % 2),
             W.serving_request(seed=k, n=16)]
    for form in ("per_box", "batched", "graph", "waves"):
        solvers = [ctuppm.Solver(ctx, p, form=form) for p in probs]
        ctx.step(solvers, form, 2)
        for s in solvers:
            s.close()
    prob = W.cloud_wind(n=32, box=16, fine_box=8, fine_region=((8, 8, 8), (24, 24, 24)))
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(1)
    s.regrid([((16, 16, 16), (31, 31, 31)), ((32, 16, 16), (47, 31, 31))])
    s.step(1, form="batched")
    s.close()


def test_library_allocates_no_device_memory(ctx):
    torch = ctx.torch
    _cycle(ctx, 0)  # warm: kernels loaded, staging buffers and the allocator's pools exist
    before = _outside_torch(torch)
    for k in range(1, 11):
        _cycle(ctx, k)  # 50 problems in all
    after = _outside_torch(torch)
    print(f"device memory outside torch: before {before} after {after} bytes", flush=True)
    assert after - before <= 4 << 20


def test_guarded_step_keeps_un_and_reports(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=24, box=12, seed=3)
    s = ctuppm.Solver(ctx, prob)
    s.set_fail_hook(1)  # the second step's update flags a failed cell, once
    s.step_guarded(3)   # accepted, rejected (U^1 kept), accepted from U^1
    ctx.torch.cuda.synchronize()
    with pytest.raises(ctuppm.Rejected):
        s.step_guarded(1)  # the host now sees the rejection
    assert s.rejections() == 1
    got = s.state()
    assert s.counters()[5] == 2
    s.step_guarded(1)  # acknowledged: accepted again
    got3 = s.state()
    s.close()
    ref2, _, _ = oracle.run_problem(prob, 2)
    ref3, _, _ = oracle.run_problem(prob, 3)
    assert np.array_equal(got, ref2) and np.array_equal(got3, ref3)


def test_checked_step_gives_up_with_un_current(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=16, box=8, seed=4)
    prob.small_pres = 100.0  # every pressure is below the floor: every step fails
    s = ctuppm.Solver(ctx, prob)
    with pytest.raises(ctuppm.Rejected):
        s.step_checked()
    got = s.state()
    cnt = s.counters()
    s.close()
    assert np.array_equal(got, prob.U0) and cnt[5] == 0 and cnt[4] > 0


def test_checked_step_redoes_a_rejected_half(ctx):
    """A failure forced in the first half step is redone as two quarter steps."""
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=24, box=12, seed=5)
    a = ctuppm.Solver(ctx, prob)
    a.set_fail_hook(0)
    assert a.step_checked() == 1  # the full step fails, its two halves pass
    got = a.state()
    a.close()
    P = oracle.params_of(prob)
    G = oracle.fill_domain(oracle.grow(prob.U0), P)
    dt = P.cfl / oracle.signal_speed(G, P)
    ref, _, _ = oracle.run(prob.U0, P, 2, dt_fixed=0.5 * dt)
    assert np.array_equal(got, ref)


def test_stage_dump_refusals(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.cloud_wind(n=32, box=16, fine_box=8, fine_region=((8, 8, 8), (24, 24, 24)))
    s = ctuppm.Solver(ctx, prob)
    s.step(1)
    with pytest.raises(ctuppm.CtuError):
        s.stage_array(0, "q", form="per_box")
    s.close()
    prob = W.kelvin_helmholtz(n=(32, 32, 16), box=(8, 8, 16), seed=1)
    ctx.set_wave_boxes(2)
    try:
        s = ctuppm.Solver(ctx, prob, form="waves")  # workspace: two scratch slots
        s.step(1)
        with pytest.raises(ctuppm.CtuError) as e:
            s.stage_array(15, "ff2", form="batched")  # the batched layout ends far past it
        assert e.value.code == ctuppm.ENOMEM
        s.stage_array(15, "ff2", form="waves")
        s.close()
    finally:
        ctx.set_wave_boxes(64)


def test_rebinding_fine_level_keeps_coarse_parity(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.cloud_wind(n=32, box=16, fine_box=8, fine_region=((8, 8, 8), (24, 24, 24)))
    s = ctuppm.Solver(ctx, prob)
    s.step(1)  # the coarse state is now in the B fabs, the fine one back in A
    before = s.state()
    s._bind(1)
    after = s.state()
    s.step(1)
    got = s.state()
    s.close()
    rc, _, _, _ = oracle.run_two_level(prob, 2)
    assert np.array_equal(before, after) and np.array_equal(got, rc)
