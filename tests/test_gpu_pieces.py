"""A step taken in pieces through the C ABI (ghost fill, dt, advance per
level, average down, reflux) against the one-call step and the oracle, a
caller's dt, and the calls the state machine must reject."""
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


def _cloud():
    return W.cloud_wind(n=32, box=16, fine_box=16, fine_region=((8, 8, 8), (24, 24, 24)), nspec=1)


def _run(ctx, prob, nsteps, pieces, form="batched", dt=None):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form=form)
    if pieces:
        s.step_in_pieces(nsteps, dt=dt)
    else:
        s.step(nsteps)
    out = (s.state(), s.state_fine() if prob.fine_boxes else None, s.counters())
    s.close()
    return out


@pytest.mark.parametrize("form", ["per_box", "batched"])
def test_single_level_pieces_equal_the_step_and_the_oracle(ctx, form):
    prob = W.kelvin_helmholtz(n=32, box=16, nspec=2)
    got, _, cnt = _run(ctx, prob, 4, True, form)
    one, _, _ = _run(ctx, prob, 4, False, "graph")
    ref, _, _ = oracle.run_problem(prob, 4)
    print(f"kh32 pieces {form}: equal to the step {np.array_equal(got, one)}, to the oracle "
          f"{np.array_equal(got, ref)}", flush=True)
    assert np.array_equal(got, one) and np.array_equal(got, ref)
    assert cnt[5] == 4 and not cnt[:5].any()


def test_rt_uneven_with_gravity_pieces(ctx):
    prob = W.rayleigh_taylor(n=48, nspec=1)
    got, _, _ = _run(ctx, prob, 3, True)
    ref, _, _ = oracle.run_problem(prob, 3)
    assert np.array_equal(got, ref)


def test_two_level_pieces_equal_the_step_and_the_oracle(ctx):
    prob = _cloud()
    gc, gf, cnt = _run(ctx, prob, 3, True)
    sc, sf, _ = _run(ctx, prob, 3, False)
    rc, rf, _, _ = oracle.run_two_level(prob, 3)
    print(f"cloud32 pieces: coarse equal to the step {np.array_equal(gc, sc)}, fine {np.array_equal(gf, sf)}; "
          f"to the oracle {np.array_equal(gc, rc)}, {np.array_equal(gf, rf)}", flush=True)
    assert np.array_equal(gc, sc) and np.array_equal(gf, sf)
    assert np.array_equal(gc, rc) and np.array_equal(gf, rf)
    assert cnt[5] == 3


def test_a_callers_dt(ctx):
    """compute_dt writes the CFL dt to a device double; advancing with half of
    it equals the oracle's step with that fixed dt.  On two levels the computed
    dt passed back gives the same state as the dt kept by the library."""
    from paper_1711_06203_amd import ctuppm
    torch = ctx.torch
    prob = W.kelvin_helmholtz(n=32, box=16)
    s = ctuppm.Solver(ctx, prob)
    d = torch.zeros(1, dtype=torch.float64, device=s.dev)
    s.fill_ghosts(0)
    s.compute_dt(out=d)
    P = oracle.params_of(prob)
    want = P.cfl / oracle.signal_speed(oracle.fill_domain(oracle.grow(prob.U0), P), P)
    dt = float(d.item())
    assert dt == want
    half = d * 0.5
    s.advance_level(0, dt=half)
    got = s.state()
    assert s.dt() == 0.5 * dt
    s.close()
    ref, _, _ = oracle.run(prob.U0, P, 1, dt_fixed=0.5 * dt)
    assert np.array_equal(got, ref)

    cloud = _cloud()
    s = ctuppm.Solver(ctx, cloud)
    d = torch.zeros(1, dtype=torch.float64, device=s.dev)
    for _ in range(2):
        s.fill_ghosts(0)
        s.compute_dt(out=d)
        s.advance_level(0, dt=d.clone())
        for _sub in range(2):
            s.fill_ghosts(1)
            s.advance_level(1)
        s.average_down()
        s.reflux()
    gc, gf = s.state(), s.state_fine()
    s.close()
    sc, sf, _ = _run(ctx, cloud, 2, False)
    assert np.array_equal(gc, sc) and np.array_equal(gf, sf)


def test_calls_out_of_order_are_rejected_and_change_nothing(ctx):
    from paper_1711_06203_amd import ctuppm
    torch = ctx.torch
    E = ctuppm.CtuError
    prob = W.kelvin_helmholtz(n=32, box=16)
    s = ctuppm.Solver(ctx, prob)
    with pytest.raises(E):
        s.advance_level(0)                     # ghosts not filled
    s.fill_ghosts(0)
    with pytest.raises(E):
        s.advance_level(0)                     # no dt
    with pytest.raises(E):
        s.fill_ghosts(1)                       # no level 1
    with pytest.raises(E):
        s.average_down()                       # one level
    with pytest.raises(E):
        s.fill_ghosts(0, form=2)               # the graph form is the whole step's
    s.compute_dt()
    s.advance_level(0)
    with pytest.raises(E):
        s.advance_level(0)                     # state changed since the fill
    got = s.state()
    s.close()
    ref, _, _ = oracle.run_problem(prob, 1)
    assert np.array_equal(got, ref)

    mol = W.kelvin_helmholtz(n=32, box=16)
    mol.scheme = 1
    s = ctuppm.Solver(ctx, mol)
    with pytest.raises(E):
        s.fill_ghosts(0)                       # method of lines: ctuppm_step only
    s.close()

    cloud = _cloud()
    s = ctuppm.Solver(ctx, cloud)
    d = torch.full((1,), 1e-3, dtype=torch.float64, device=s.dev)
    with pytest.raises(E):
        s.fill_ghosts(1)                       # before the coarse advance
    with pytest.raises(E):
        s.advance_level(1)
    with pytest.raises(E):
        s.fill_ghosts(0, form="per_box")       # two levels: batched only
    s.fill_ghosts(0)
    s.compute_dt()
    s.advance_level(0)
    for bad in (lambda: s.step(), lambda: s.tag(0.1), lambda: s.fill_ghosts(0), lambda: s.compute_dt(),
                lambda: s.advance_level(0), lambda: s.average_down(), lambda: s.reflux(),
                lambda: s.advance_level(1),                 # fine ghosts not filled
                lambda: s.advance_level(1, dt=d)):          # the fine level takes half the coarse dt
        with pytest.raises(E):
            bad()
    for _sub in range(2):
        s.fill_ghosts(1)
        s.advance_level(1)
    with pytest.raises(E):
        s.fill_ghosts(1)                       # a third substep
    with pytest.raises(E):
        s.reflux()                             # before averaging down
    s.average_down()
    with pytest.raises(E):
        s.average_down()
    s.reflux()
    gc, gf = s.state(), s.state_fine()
    s.step(1)                                  # a whole step is allowed again
    s.close()
    rc, rf, _, _ = oracle.run_two_level(cloud, 1)
    assert np.array_equal(gc, rc) and np.array_equal(gf, rf)
