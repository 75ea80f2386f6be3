"""The waves form: batched launches over waves of consecutive boxes that share
as many stage scratch slots (the workspace scales with the wave).  Bitwise
the oracle's results for every wave size, scheme and variant, several
problems stepped together, steps in pieces, and a 256^3 box set in waves of
16 (sampled); two levels are refused."""
import ctypes

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
    c.set_wave_boxes(64)
    c.close()


def _kh(**kw):
    prob = W.kelvin_helmholtz(n=(40, 36, 20), box=(16, 16, 20), nspec=2)  # 9 boxes, ragged tails
    for k, v in kw.items():
        setattr(prob, k, v)
    return prob


def _run(ctx, prob, nsteps, pieces=False):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form="waves")
    if pieces:
        s.step_in_pieces(nsteps)
    else:
        s.step(nsteps)
    out, ws = s.state(), s.ws.numel()
    s.close()
    return out, ws


@pytest.mark.parametrize("wave", [1, 2, 4, 9, 64])
def test_wave_sizes(ctx, wave):
    from paper_1711_06203_amd import ctuppm
    ctx.set_wave_boxes(wave)
    prob = _kh()
    got, ws = _run(ctx, prob, 4)
    ref, _, _ = oracle.run_problem(prob, 4)
    assert np.array_equal(got, ref)
    # the workspace holds min(wave, boxes) scratch slots, not the whole level's
    s = ctuppm.Solver(ctx, prob, form="per_box")
    b = ctypes.c_size_t()
    ctx.call("ctuppm_workspace_bytes", s.pid, ctuppm.FORM_BATCHED, ctypes.byref(b))
    s.close()
    if wave < 9:
        assert ws < b.value


@pytest.mark.parametrize("variant", [dict(scheme=2), dict(scheme=1, riemann=1, limiter=1), dict(steepen=1)])
def test_variants_in_waves_of_four(ctx, variant):
    ctx.set_wave_boxes(4)
    prob = _kh(**variant)
    got, _ = _run(ctx, prob, 3)
    ref, _, _ = oracle.run_problem(prob, 3)
    assert np.array_equal(got, ref), variant


def test_problems_stepped_together_and_pieces(ctx):
    from paper_1711_06203_amd import ctuppm
    ctx.set_wave_boxes(3)
    a = W.rayleigh_taylor(n=(32, 16, 48), seed=11, nspec=1)
    b = W.kelvin_helmholtz(n=(24, 20, 16), box=(16, 16, 16), nspec=1)
    sa, sb = ctuppm.Solver(ctx, a, form="waves"), ctuppm.Solver(ctx, b, form="waves")
    ctx.step([sa, sb], form="waves", nsteps=3)
    ga, gb = sa.state(), sb.state()
    sa.close()
    sb.close()
    ra, _, _ = oracle.run_problem(a, 3)
    rb, _, _ = oracle.run_problem(b, 3)
    assert np.array_equal(ga, ra) and np.array_equal(gb, rb)
    got, _ = _run(ctx, a, 2, pieces=True)
    ref, _, _ = oracle.run_problem(a, 2)
    assert np.array_equal(got, ref)


def test_two_levels_are_refused(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.cloud_wind(n=32, box=16, fine_box=16, fine_region=((8, 8, 8), (24, 24, 24)))
    s = ctuppm.Solver(ctx, prob)
    with pytest.raises(ctuppm.CtuError):
        s.step(1, form="waves")
    s.close()


@pytest.mark.slow
def test_kh256_in_waves_of_16_sampled(ctx):
    from paper_1711_06203_amd import ctuppm
    ctx.set_wave_boxes(16)
    prob = W.kelvin_helmholtz(n=256, box=64)
    s = ctuppm.Solver(ctx, prob, form="waves")
    s.step(1)
    got = s.state()
    dt_gpu = s.dt()
    s.close()
    ctx.torch.cuda.empty_cache()
    P = oracle.params_of(prob)
    G = oracle.fill_domain(oracle.grow(prob.U0), P)
    dt = P.cfl / oracle.signal_speed(G, P)
    assert dt_gpu == dt
    rng = np.random.default_rng(16)
    cells = [tuple(int(v) for v in rng.integers(256, size=3)) for _ in range(150)]
    for w in range(4):  # the first and last boxes of each wave
        for bi in (16 * w, 16 * w + 15):
            lo, hi = prob.boxes[bi]
            cells += [tuple(lo), tuple(hi)]
    want = oracle.sample_step(G, P, dt, cells)
    for c, wv in zip(cells, want):
        assert np.array_equal(got[:, c[2], c[1], c[0]], wv), c
