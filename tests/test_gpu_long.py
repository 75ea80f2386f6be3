"""The full-size workloads for their whole length: KH 256^3 for 1000 steps
(ten times its configured 100), RT 384^3 on 1436 uneven boxes for its 200
steps, the two-level cloud for its 100 coarse steps.  No floors, fall-backs or
failed cells; every value finite; on the periodic KH domain the conserved
totals stay those of the initial state to round-off, and the mass of the
walled RT domain likewise."""
import math

import numpy as np
import pytest

from paper_1711_06203_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


def _totals(U):
    return [math.fsum(U[m].ravel()) for m in range(U.shape[0])]


def _run(ctx, prob, steps, chunk=100):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form="graph")
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        s.step(k)
        done += k
        print(f"{prob.name}: {done} steps, dt {s.dt():.3e}", flush=True)
    out = (s.state(), s.state_fine() if prob.fine_boxes else None, s.counters())
    s.close()
    ctx.torch.cuda.empty_cache()
    return out


def test_kh256_thousand_steps(ctx):
    prob = W.kelvin_helmholtz(n=256, box=64)
    U, _, cnt = _run(ctx, prob, 1000)
    assert np.isfinite(U).all()
    assert not cnt[:5].any() and cnt[5] == 1000
    t0, t1 = _totals(prob.U0), _totals(U)
    scale = math.fsum(np.abs(prob.U0[4]).ravel())  # the energy sets the round-off scale of every total
    for m in range(5):
        assert abs(t1[m] - t0[m]) <= 1e-12 * scale, (m, t0[m], t1[m])


def test_rt384_two_hundred_steps(ctx):
    prob = W.rayleigh_taylor(n=384)
    U, _, cnt = _run(ctx, prob, 200, chunk=50)
    assert np.isfinite(U).all()
    assert not cnt[:5].any() and cnt[5] == 200
    m0, m1 = math.fsum(prob.U0[0].ravel()), math.fsum(U[0].ravel())
    assert abs(m1 - m0) <= 1e-12 * m0


def test_cloud256_hundred_coarse_steps(ctx):
    prob = W.cloud_wind(n=256, box=64, fine_box=32)
    Uc, Uf, cnt = _run(ctx, prob, 100, chunk=25)
    assert np.isfinite(Uc).all() and np.isfinite(Uf).all()
    assert not cnt[:5].any() and cnt[5] == 100
    assert Uc[0].min() > 0.0 and Uf[0].min() > 0.0


def test_kh256_hundred_steps_same_in_every_form(ctx):
    """The configured 100 KH steps give bitwise the same state in the graph,
    batched, per-box and waves forms (the graph form's state after 100 steps
    is the one the other forms must reproduce)."""
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=256, box=64)
    ref = None
    ctx.set_wave_boxes(16)
    for form in ("graph", "batched", "per_box", "waves"):
        s = ctuppm.Solver(ctx, prob, form=form)
        s.step(100)
        got = s.state()
        s.close()
        ctx.torch.cuda.empty_cache()
        print(f"kh256 100 steps, {form}: bitwise {ref is None or np.array_equal(got, ref)}", flush=True)
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got, ref), form
    ctx.set_wave_boxes(64)
