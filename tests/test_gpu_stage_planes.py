"""Per-stage launch shapes: the planes each work unit of a stage marches
through (ctuppm_set_stage_planes) change which block computes which cell,
never a cell's arithmetic, so every setting gives the oracle's bits; the
per-stage autotuner only times."""
import numpy as np
import pytest

import oracle
from paper_1711_06203_amd import workloads as W

pytestmark = pytest.mark.gpu

DEFAULTS = {"cons2prim_cfl": 2, "trace_xyz": 4, "trans1_xyz": 1, "riemann_x": 1, "riemann_y": 1, "riemann_z": 1,
            "trans2_x": 1, "trans2_y": 1, "trans2_z": 1, "update": 1, "recon_x": 1, "cons2prim": 2}


@pytest.fixture(scope="module")
def ctx():
    from paper_1711_06203_amd import ctuppm
    c = ctuppm.Context()
    yield c
    c.close()


def _restore(ctx):
    for st, p in DEFAULTS.items():
        ctx.set_stage_planes(st, p)


def _run(ctx, prob, steps, form="graph"):
    from paper_1711_06203_amd import ctuppm
    s = ctuppm.Solver(ctx, prob, form=form)
    s.step(steps)
    out = [s.state()] + (s.state_patches() if prob.fine_boxes else [])
    s.close()
    return out


def test_defaults_and_refusals(ctx):
    from paper_1711_06203_amd import ctuppm
    assert ctx.stage_planes("trace_xyz")[0] == 4 and ctx.stage_planes("cons2prim_cfl")[0] == 2
    assert ctx.stage_planes("trans1_xyz")[0] == 1
    # stages over the same work region share one group
    assert ctx.stage_planes("trans1_xyz")[1] == ctx.stage_planes("flatten")[1]
    assert ctx.stage_planes("trace_xyz")[1] != ctx.stage_planes("trans1_xyz")[1]
    for bad in (("fill", 2), ("dt", 2), ("trace_xyz", 0), ("trace_xyz", 65)):
        with pytest.raises(ctuppm.CtuError):
            ctx.set_stage_planes(*bad)
    assert ctx.stage_planes("trace_xyz")[0] == 4


@pytest.mark.parametrize("setting", [
    {"trace_xyz": 1},
    {"trace_xyz": 8, "trans1_xyz": 3, "riemann_y": 5, "trans2_z": 2, "update": 7, "cons2prim_cfl": 1},
])
def test_any_setting_gives_the_oracle_bits(ctx, setting):
    prob = W.kelvin_helmholtz(n=(40, 36, 28), box=(16, 16, 20), nspec=2, seed=9)
    try:
        for st, p in setting.items():
            ctx.set_stage_planes(st, p)
        got = _run(ctx, prob, 3)
        got_batched = _run(ctx, prob, 3, form="batched")
    finally:
        _restore(ctx)
    ref, _, _ = oracle.run_problem(prob, 3)
    assert np.array_equal(got[0], ref) and np.array_equal(got_batched[0], ref)


def test_two_level_and_mol_under_deep_units(ctx):
    cloud = W.cloud_wind(n=32, box=16, fine_box=8, fine_region=((10, 10, 10), (22, 22, 22)), nspec=1)
    mol = W.kelvin_helmholtz(n=(32, 24, 24), box=(16, 12, 24), nspec=1, seed=2)
    mol.scheme = 1
    try:
        for st in ("trace_xyz", "trans1_xyz", "recon_x", "trans2_x"):
            ctx.set_stage_planes(st, 6)
        g_cloud = _run(ctx, cloud, 3)
        g_mol = _run(ctx, mol, 3)
    finally:
        _restore(ctx)
    rc, rf, _, _ = oracle.run_two_level(cloud, 3)
    assert np.array_equal(g_cloud[0], rc) and np.array_equal(g_cloud[1], rf)
    ref, _, _ = oracle.run_problem(mol, 3)
    assert np.array_equal(g_mol[0], ref)


def test_stage_tuner_picks_per_group_and_keeps_the_bits(ctx):
    from paper_1711_06203_amd import autotune, ctuppm
    prob = W.kelvin_helmholtz(n=(48, 48, 48), box=(24, 24, 24), seed=4)
    s = ctuppm.Solver(ctx, prob)
    try:
        out = autotune.tune_stages(ctx, [s], candidates=(1, 2, 4), steps=2, cache=None)
        ran = set(out["planes"])
        assert {"trace_xyz", "trans1_xyz", "riemann_x", "trans2_z", "update"} <= ran
        assert all(p in (1, 2, 4) for p in out["planes"].values()) or out["planes"] == {
            st: ctx.stage_planes(st)[0] for st in out["planes"]}
        for st, p in out["planes"].items():
            assert ctx.stage_planes(st)[0] == p
        print(f"stage planes chosen: {out['planes']}, {out['start_ms_per_step']:.3f} -> {out['ms_per_step']:.3f} ms",
              flush=True)
        s.upload(prob.U0)
        s.step(3)
        got = s.state()
    finally:
        s.close()
        _restore(ctx)
    ref, _, _ = oracle.run_problem(prob, 3)
    assert np.array_equal(got, ref)
