"""ctuppm_step_static (the step for callers that cannot allocate: stage
scratch in the library's static device array) against ctuppm_step in the
batched form, called through the C ABI: bitwise the same states on two calls
in a row, the second problem smaller than the first, and nothing allocated."""
import ctypes

import numpy as np
import pytest

from paper_1711_06203_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


def _pair(ctx, prob, steps):
    """The same problem stepped by ctuppm_step (batched) and ctuppm_step_static."""
    from paper_1711_06203_amd import ctuppm
    torch = ctx.torch
    a = ctuppm.Solver(ctx, prob, form="batched")
    a.step(steps)
    want = a.state()
    a.close()
    b = ctuppm.Solver(ctx, prob, form="per_box")  # a workspace without the level's scratch
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(steps):
        ctx.call("ctuppm_step_static", b.pid)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    got = b.state()
    b.close()
    return got, want, free0 - free1


def test_static_step_equals_batched_twice(ctx):
    big = W.kelvin_helmholtz(n=(32, 24, 16), box=(16, 24, 16), seed=7, nspec=1)
    got, want, grew = _pair(ctx, big, 3)
    assert np.array_equal(got, want) and grew == 0
    small = W.serving_request(seed=11, n=16)
    small.scheme = 1  # the method of lines uses the workspace's stage fabs
    got, want, grew = _pair(ctx, small, 2)
    assert np.array_equal(got, want) and grew == 0


def test_static_step_refuses_what_does_not_fit(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=(64, 64, 32), box=(32, 32, 32), seed=1)  # 4 boxes: ~130 MB of scratch
    s = ctuppm.Solver(ctx, prob, form="per_box")
    with pytest.raises(ctuppm.CtuError) as e:
        ctx.call("ctuppm_step_static", s.pid)
    assert e.value.code == ctuppm.EINVAL
    s.close()
