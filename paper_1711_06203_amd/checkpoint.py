"""Checkpoint and resume of a problem resident on the GPU.

A checkpoint is one ``.npz`` file: the valid cells of the current state of
every level and the problem's description as a JSON string (no pickled
objects; it loads with ``allow_pickle=False``).  The valid cells describe the
device state completely -- every step refills the ghost cells first and takes
dt from the state (or the fixed dt, which is saved) -- so a run resumed from
a checkpoint continues bitwise as the uninterrupted one.  The library's
counters (floors, fall-backs, steps) start again from zero; the number of
steps taken before the checkpoint is kept in the description.
"""
from __future__ import annotations

import json
from typing import Optional, Sequence, Tuple

import numpy as np

from . import workloads as W

FORMAT = 1

# Problem fields saved as they are (tuples become lists in JSON).
_FIELDS = ("name", "n", "gamma", "bc_lo", "bc_hi", "cfl", "grav_z", "inflow", "prob_lo", "prob_hi", "steps",
           "small_dens", "small_pres", "nspec", "inflow_X", "scheme", "riemann", "limiter", "steepen")
_TUPLES = ("n", "bc_lo", "bc_hi", "inflow", "prob_lo", "prob_hi", "inflow_X")


def _plain(v):
    if isinstance(v, (tuple, list)):
        return [_plain(x) for x in v]
    if isinstance(v, np.generic):
        return v.item()
    return v


def save(path: str, prob: W.Problem, U: np.ndarray, U_fine: Optional[np.ndarray] = None,
         fine_lo: Optional[Sequence[int]] = None, fine_boxes: Optional[Sequence[W.Box]] = None,
         steps_taken: int = 0, fixed_dt: Optional[float] = None) -> None:
    """Write the state U (5 + nspec, nz, ny, nx) of `prob`'s level 0 and, for a
    two-level problem, the fine rectangle's state starting at fine index
    `fine_lo` with its boxes."""
    meta = {k: _plain(getattr(prob, k)) for k in _FIELDS}
    meta["format"] = FORMAT
    meta["boxes"] = [[list(map(int, lo)), list(map(int, hi))] for lo, hi in prob.boxes]
    meta["steps_taken"] = int(steps_taken)
    meta["fixed_dt"] = None if not fixed_dt else float(fixed_dt)
    nv = 5 + int(prob.nspec)
    if U.shape != (nv,) + tuple(prob.n[::-1]):
        raise ValueError(f"state shape {U.shape} does not match the problem ({nv}, {prob.n[::-1]})")
    arrays = {"U": np.ascontiguousarray(U, dtype=np.float64)}
    if U_fine is not None:
        if fine_lo is None or not fine_boxes:
            raise ValueError("a fine state needs its first index and its boxes")
        meta["fine_lo"] = [int(v) for v in fine_lo]
        meta["fine_boxes"] = [[list(map(int, lo)), list(map(int, hi))] for lo, hi in fine_boxes]
        arrays["U_fine"] = np.ascontiguousarray(U_fine, dtype=np.float64)
    np.savez(path, meta=np.array(json.dumps(meta)), **arrays)


def load(path: str) -> Tuple[W.Problem, dict]:
    """The problem to resume (its initial state is the saved state) and the
    saved description."""
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        if meta.get("format") != FORMAT:
            raise ValueError(f"{path}: checkpoint format {meta.get('format')} is not {FORMAT}")
        U = np.array(z["U"], dtype=np.float64)
        U_fine = np.array(z["U_fine"], dtype=np.float64) if "U_fine" in z.files else None
    kw = {k: (tuple(meta[k]) if k in _TUPLES else meta[k]) for k in _FIELDS}
    prob = W.Problem(U0=U, boxes=[(tuple(lo), tuple(hi)) for lo, hi in meta["boxes"]], **kw)
    if U_fine is not None:
        prob.U0_fine = U_fine
        prob.fine_lo = tuple(meta["fine_lo"])
        prob.fine_boxes = [(tuple(lo), tuple(hi)) for lo, hi in meta["fine_boxes"]]
    return prob, meta
