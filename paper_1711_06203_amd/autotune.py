"""Autotuners of the launch shapes of the batched form.

``tune``: one setting for every stage (``ctuppm_set_tuning2``): blocks per
CU of the launches (0 = one block per work unit, else a persistent grid of
that many blocks per CU walking the units), the z planes a work unit marches
through, and the rows per tile the units of a plane are grouped into.

``tune_stages``: the planes per work unit of each stage on its own
(``ctuppm_set_stage_planes``; stages over the same work region share one
setting).  Every stage group is timed at every candidate from the library's
per-stage timing of whole steps, each group takes its fastest, and the
combination is kept only if a timed step confirms it.

Every choice gives bitwise the same results (each cell's arithmetic is
fixed), so the tuners only time: a few event-timed eager steps per candidate
on the caller's problems.  Choices are cached in a JSON file keyed by the
workload's box-size signature.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

from . import ctuppm

# (blocks_per_cu, zseg, ytile)
DEFAULT_CANDIDATES: Tuple[Tuple[int, int, int], ...] = ((0, 1, 0), (0, 2, 0), (0, 1, 4), (0, 1, 8), (0, 2, 8),
                                                        (0, 4, 8), (16, 1, 0), (16, 2, 8))
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def signature(solvers: Sequence[ctuppm.Solver]) -> str:
    """Box-size histogram of the problems stepped together."""
    hist: Dict[str, int] = {}
    for s in solvers:
        for lo, hi in s.prob.boxes:
            key = "x".join(str(hi[d] - lo[d] + 1) for d in range(3))
            hist[key] = hist.get(key, 0) + 1
    return ";".join(f"{k}:{v}" for k, v in sorted(hist.items()))


def _time_steps(ctx: ctuppm.Context, solvers, steps: int) -> float:
    ctx.step(solvers, "batched", 1)
    ctx.torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.step(solvers, "batched", steps)
    ctx.set_timing(False)
    st = ctx.stage_times()
    return sum(ms for ms, n in st.values()) / steps


def tune(ctx: ctuppm.Context, solvers: Sequence[ctuppm.Solver], candidates: Iterable[Tuple[int, ...]] = DEFAULT_CANDIDATES,
         steps: int = 3, cache: Optional[str] = CACHE, use_cache: bool = True) -> dict:
    """Pick (blocks_per_cu, zseg, ytile) for these problems; applies and returns it.

    The problems are advanced by the timing steps (1 + steps per candidate),
    so callers tune on a copy or before loading the real initial state."""
    key = signature(solvers)
    db = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    if use_cache and key in db:
        best = db[key]
        ctx.set_tuning(best["blocks_per_cu"], best["zseg"], 1, best.get("ytile", 0))
        return dict(best, cached=True)
    trials: List[dict] = []
    for cand in candidates:
        bpc, zseg = cand[0], cand[1]
        ytile = cand[2] if len(cand) > 2 else 0
        ctx.set_tuning(bpc, zseg, 1, ytile)
        ms = _time_steps(ctx, solvers, steps)
        trials.append({"blocks_per_cu": bpc, "zseg": zseg, "ytile": ytile, "ms_per_step": ms})
    best = min(trials, key=lambda t: t["ms_per_step"])
    ctx.set_tuning(best["blocks_per_cu"], best["zseg"], 1, best["ytile"])
    out = dict(best, trials=trials, signature=key, when=time.strftime("%Y-%m-%dT%H:%M:%S"))
    if cache:
        db[key] = {"blocks_per_cu": best["blocks_per_cu"], "zseg": best["zseg"], "ytile": best["ytile"],
                   "ms_per_step": best["ms_per_step"]}
        try:
            with open(cache, "w") as f:
                json.dump(db, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return dict(out, cached=False)


STAGE_CANDIDATES: Tuple[int, ...] = (1, 2, 4, 8)


def _stage_ms(ctx: ctuppm.Context, solvers, steps: int) -> Dict[str, float]:
    """Per-stage milliseconds per step of eager batched steps (one warm-up step
    first: it rebuilds work lists after a tuning change)."""
    ctx.step(solvers, "batched", 1)
    ctx.torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.step(solvers, "batched", steps)
    ctx.set_timing(False)
    return {k: ms / steps for k, (ms, n) in ctx.stage_times().items() if n}


def _load(cache: Optional[str]) -> dict:
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}
    return {}


def tune_stages(ctx: ctuppm.Context, solvers: Sequence[ctuppm.Solver],
                candidates: Iterable[int] = STAGE_CANDIDATES, steps: int = 3, cache: Optional[str] = CACHE,
                use_cache: bool = True) -> dict:
    """Pick the planes per work unit of every stage group for these problems;
    applies and returns {"planes": {stage: planes}, ...}.  The problems are
    advanced by the timing steps."""
    key = "stages:" + signature(solvers)
    db = _load(cache)
    if use_cache and key in db:
        for st, p in db[key]["planes"].items():
            ctx.set_stage_planes(st, p)
        return dict(db[key], cached=True)
    start = _stage_ms(ctx, solvers, steps)
    groups: Dict[int, List[str]] = {}
    before: Dict[str, int] = {}
    for st in start:
        try:
            p, g = ctx.stage_planes(st)
        except ctuppm.CtuError:
            continue  # no work units (ghost fill, boundaries, dt, commit)
        groups.setdefault(g, []).append(st)
        before[st] = p
    lead = {g: sts[0] for g, sts in groups.items()}
    trials: Dict[int, Dict[str, float]] = {}
    for p in candidates:
        for g in groups:
            ctx.set_stage_planes(lead[g], p)
        trials[p] = _stage_ms(ctx, solvers, steps)
    best: Dict[int, int] = {}
    for g, sts in groups.items():
        best[g] = min(trials, key=lambda p: sum(trials[p].get(st, 0.0) for st in sts))
    for g, p in best.items():
        ctx.set_stage_planes(lead[g], p)
    tuned = sum(_stage_ms(ctx, solvers, steps).values())
    base_total = sum(start.values())
    planes = {st: best[g] for g, sts in groups.items() for st in sts}
    if tuned > base_total:  # the groups interact through the caches: keep the starting setting
        for st, p in before.items():
            ctx.set_stage_planes(st, p)
        planes = dict(before)
    out = {"planes": planes, "ms_per_step": min(tuned, base_total), "start_ms_per_step": base_total,
           "trials": {str(p): t for p, t in trials.items()}, "signature": key,
           "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    if cache:
        db[key] = {"planes": planes, "ms_per_step": out["ms_per_step"]}
        try:
            with open(cache, "w") as f:
                json.dump(db, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return dict(out, cached=False)

