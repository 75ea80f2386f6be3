"""The per-stage autotuner's host logic against a modelled context (no GPU):
each stage group takes the candidate that minimises its stages' summed time,
stages of one group share the choice, a combination that times slower than
the starting setting is dropped, and choices are cached per signature."""
import types

from paper_1711_06203_amd import autotune, ctuppm

# stage -> group (stages of one group share their setting)
GROUPS = {"cons2prim_cfl": 1, "trace_xyz": 9, "trans1_xyz": 2, "flatten": 2, "riemann_x": 3, "update": 0}
BEST = {"cons2prim_cfl": 2, "trace_xyz": 4, "trans1_xyz": 1, "flatten": 8, "riemann_x": 1, "update": 1}


class ModelCtx:
    """Stage time = 1 + (log2 planes - log2 best)^2 (+ an interaction penalty
    when every group is away from 1 plane, to exercise the fall-back)."""

    def __init__(self, interaction=0.0):
        self.planes = {g: 1 for g in set(GROUPS.values())}
        self.interaction = interaction
        self.timing = False
        self.acc = {}
        self.torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))

    def stage_planes(self, st):
        if st not in GROUPS:
            raise ctuppm.CtuError(f"stage {st} has no work units", ctuppm.EINVAL)
        g = GROUPS[st]
        return self.planes[g], g

    def set_stage_planes(self, st, p):
        self.planes[GROUPS[st]] = int(p)

    def set_timing(self, on):
        self.timing = bool(on)
        if on:
            self.acc = {}

    def _ms(self, st):
        lg = {1: 0, 2: 1, 4: 2, 8: 3}
        t = 1.0 + (lg[self.planes[GROUPS[st]]] - lg[BEST[st]]) ** 2
        if self.interaction and all(p > 1 for p in self.planes.values()):
            t += self.interaction
        return t

    def step(self, solvers, form, n):
        if not self.timing:
            return
        for st in list(GROUPS) + ["fill"]:
            ms = 0.5 if st == "fill" else self._ms(st)
            a = self.acc.get(st, (0.0, 0))
            self.acc[st] = (a[0] + ms * n, a[1] + n)

    def stage_times(self):
        return dict(self.acc)


def _solver():
    return types.SimpleNamespace(prob=types.SimpleNamespace(boxes=[((0, 0, 0), (63, 63, 63))] * 2))


def test_groups_take_their_fastest_candidate():
    ctx = ModelCtx()
    out = autotune.tune_stages(ctx, [_solver()], candidates=(1, 2, 4, 8), steps=2, cache=None)
    assert "fill" not in out["planes"]
    assert out["planes"]["trace_xyz"] == 4 and out["planes"]["cons2prim_cfl"] == 2
    assert out["planes"]["riemann_x"] == 1 and out["planes"]["update"] == 1
    # trans1_xyz (best 1) and flatten (best 8) share a group: the summed time is
    # 1 + 10 at 1 plane, 2 + 5 at 2, 5 + 2 at 4, 10 + 1 at 8, so 2 and 4 tie and
    # the first candidate reached wins
    assert out["planes"]["trans1_xyz"] == out["planes"]["flatten"] == 2
    assert ctx.planes[9] == 4 and ctx.planes[2] == 2
    assert out["ms_per_step"] <= out["start_ms_per_step"]


def test_a_slower_combination_is_dropped():
    ctx = ModelCtx(interaction=100.0)
    ctx.planes[9] = 4  # a starting setting away from the defaults of the model
    out = autotune.tune_stages(ctx, [_solver()], candidates=(1, 2, 4, 8), steps=1, cache=None)
    assert out["ms_per_step"] == out["start_ms_per_step"]
    assert ctx.planes[9] == 4 and ctx.planes[1] == 1 and ctx.planes[2] == 1


def test_choices_are_cached_per_signature(tmp_path):
    cache = str(tmp_path / "tuning.json")
    ctx = ModelCtx()
    first = autotune.tune_stages(ctx, [_solver()], steps=1, cache=cache)
    assert not first["cached"]
    other = ModelCtx()
    second = autotune.tune_stages(other, [_solver()], steps=1, cache=cache)
    assert second["cached"] and second["planes"] == first["planes"]
    assert other.planes == ctx.planes
    elsewhere = autotune.tune_stages(ModelCtx(), [types.SimpleNamespace(prob=types.SimpleNamespace(
        boxes=[((0, 0, 0), (31, 31, 31))]))], steps=1, cache=cache)
    assert not elsewhere["cached"]
