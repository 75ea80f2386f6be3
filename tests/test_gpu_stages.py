"""Stage-by-stage parity: after one step, every intermediate array of a box
(primitives, flattening, traced states, normal fluxes, both transverse-stage
fluxes, final fluxes), read back through ctuppm_debug_stage, equals the
oracle's stage dump for the same box on the same inputs, bit for bit, over
the region each stage defines.  A full-step mismatch would show here which
stage it starts in."""
import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import workloads as W

pytestmark = pytest.mark.gpu

NG = 4


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


def _oracle_stages(prob, box):
    P = oracle.params_of(prob)
    G = oracle.fill_domain(oracle.grow(prob.U0), P)
    dt = P.cfl / oracle.signal_speed(G, P)
    lo, hi = box
    sub = np.ascontiguousarray(G[:, lo[2]:hi[2] + 1 + 2 * NG, lo[1]:hi[1] + 1 + 2 * NG, lo[0]:hi[0] + 1 + 2 * NG])
    Pb = oracle.with_faces(P, [-lo[d] for d in range(3)], [prob.n[d] - lo[d] for d in range(3)])
    _, _, st = oracle.advance_box(sub, Pb, dt, stages=True)
    return st, dt


def _compare(s, prob, b, form="batched"):
    want, dt = _oracle_stages(prob, prob.boxes[b])
    assert s.dt() == dt
    checked = 0
    for name in s.STAGE_ARRAYS:
        got = s.stage_array(b, name, form=form)
        ref = want[name]
        assert got.shape == ref.shape, (name, got.shape, ref.shape)
        mask = np.isfinite(ref)
        assert mask.any(), name
        bad = np.argwhere((got != ref) & mask)
        assert bad.size == 0, (name, bad[:3].tolist(), got[tuple(bad[0])], ref[tuple(bad[0])])
        checked += int(mask.sum())
    return checked


@pytest.mark.parametrize("b", [0, 5])
def test_kh_species_every_stage(ctx, b):
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=32, box=16, nspec=2)
    s = ctuppm.Solver(ctx, prob, form="batched")
    s.step(1)
    n = _compare(s, prob, b)
    s.close()
    assert n > 500_000  # values compared over the 20 arrays


def test_walls_and_gravity_every_stage(ctx):
    """A box of the RT problem on the lower reflecting wall and one on the
    upper: the wall-face states and fluxes included."""
    from paper_1711_06203_amd import ctuppm
    prob = W.rayleigh_taylor(n=(32, 16, 48), seed=11, nspec=1)
    lower = min(range(len(prob.boxes)), key=lambda i: prob.boxes[i][0][2])
    upper = max(range(len(prob.boxes)), key=lambda i: prob.boxes[i][1][2])
    assert prob.boxes[lower][0][2] == 0 and prob.boxes[upper][1][2] == prob.n[2] - 1
    s = ctuppm.Solver(ctx, prob, form="graph")
    s.step(1)
    for b in (lower, upper):
        _compare(s, prob, b, form="graph")
    s.close()


def test_per_box_form_keeps_the_last_box(ctx):
    from paper_1711_06203_amd import ctuppm
    prob = W.kelvin_helmholtz(n=(24, 16, 16), box=(8, 16, 16))
    prob.riemann, prob.limiter = 1, 1
    s = ctuppm.Solver(ctx, prob, form="per_box")
    s.step(1)
    _compare(s, prob, len(prob.boxes) - 1, form="per_box")
    s.close()


def test_waves_form_keeps_each_slots_last_box(ctx):
    """Waves of three boxes: the last wave's boxes left their arrays in the
    three scratch slots."""
    from paper_1711_06203_amd import ctuppm
    ctx.set_wave_boxes(3)
    prob = W.kelvin_helmholtz(n=(40, 36, 20), box=(16, 16, 20), nspec=1)  # 9 boxes
    s = ctuppm.Solver(ctx, prob, form="waves")
    s.step(1)
    for b in (6, 7, 8):
        _compare(s, prob, b, form="waves")
    s.close()
    ctx.set_wave_boxes(64)
