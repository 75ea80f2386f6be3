"""Checkpoint files (host side): every field of a problem survives a save and
load, the file holds no pickled objects, and a wrong format is refused."""
import json

import numpy as np
import pytest

from paper_1711_06203_amd import checkpoint, workloads as W


def _same_problem(a, b):
    for k in checkpoint._FIELDS:
        va, vb = getattr(a, k), getattr(b, k)
        assert (tuple(va) if isinstance(va, (list, tuple)) else va) == \
            (tuple(vb) if isinstance(vb, (list, tuple)) else vb), k
    assert [tuple(map(tuple, x)) for x in a.boxes] == [tuple(map(tuple, x)) for x in b.boxes]


def test_single_level_round_trip(tmp_path):
    prob = W.rayleigh_taylor(n=(16, 16, 32), seed=3, nspec=2)
    prob.scheme, prob.riemann, prob.limiter = 1, 1, 1
    U = prob.U0 + 1e-3
    p = str(tmp_path / "rt.npz")
    checkpoint.save(p, prob, U, steps_taken=7, fixed_dt=2.5e-3)
    got, meta = checkpoint.load(p)
    _same_problem(prob, got)
    assert np.array_equal(got.U0, U) and got.U0.dtype == np.float64
    assert meta["steps_taken"] == 7 and meta["fixed_dt"] == 2.5e-3
    assert got.fine_boxes is None
    with np.load(p, allow_pickle=False) as z:   # nothing pickled in the file
        assert sorted(z.files) == ["U", "meta"]


def test_two_level_round_trip(tmp_path):
    prob = W.cloud_wind(n=32, box=16, fine_box=16, fine_region=((8, 8, 8), (24, 24, 24)), nspec=1)
    lo = (18, 16, 16)
    boxes = W.regular_boxes((28, 32, 32), (16, 16, 16), origin=lo)
    Uf = np.ones((6, 32, 32, 28))
    p = str(tmp_path / "cloud.npz")
    checkpoint.save(p, prob, prob.U0, Uf, lo, boxes, steps_taken=3)
    got, meta = checkpoint.load(p)
    _same_problem(prob, got)
    assert got.fine_lo == lo and got.fine_boxes == [tuple(map(tuple, b)) for b in boxes]
    assert np.array_equal(got.U0_fine, Uf) and meta["fixed_dt"] is None


def test_bad_inputs_are_refused(tmp_path):
    prob = W.sod(n=(16, 4, 4))
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "a.npz"), prob, prob.U0[:, :2])          # wrong shape
    with pytest.raises(ValueError):
        checkpoint.save(str(tmp_path / "b.npz"), prob, prob.U0, prob.U0)         # fine state, no geometry
    p = str(tmp_path / "c.npz")
    checkpoint.save(p, prob, prob.U0)
    with np.load(p, allow_pickle=False) as z:
        meta = json.loads(str(z["meta"]))
        U = np.array(z["U"])
    meta["format"] = 99
    np.savez(p, meta=np.array(json.dumps(meta)), U=U)
    with pytest.raises(ValueError):
        checkpoint.load(p)
