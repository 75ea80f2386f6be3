"""The C-ABI library builds for gfx950, loads, and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ctuppm.h")).read()
    return sorted(set(re.findall(r"\b(ctuppm_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1711_06203_amd import ctuppm
    path = ctuppm.LIB_PATH
    if not os.path.exists(path):
        pytest.skip("library not built (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(ctuppm.EXPORTED) <= set(names)


def test_host_only_calls_without_gpu():
    from paper_1711_06203_amd import ctuppm
    if not os.path.exists(ctuppm.LIB_PATH):
        pytest.skip("library not built")
    L = ctuppm.lib()
    b = ctuppm.Box()
    b.lo[:] = [0, 0, 0]
    b.hi[:] = [63, 31, 15]
    e = ctypes.c_longlong()
    assert L.ctuppm_fab_elems(ctypes.byref(b), 0, ctypes.byref(e)) == 0
    assert e.value == 5 * 72 * 40 * 24
    assert L.ctuppm_fab_elems(ctypes.byref(b), 13, ctypes.byref(e)) == 0
    assert e.value == 18 * 72 * 40 * 24
    assert L.ctuppm_fab_elems(ctypes.byref(b), 17, ctypes.byref(e)) == ctuppm.EINVAL
    b.hi[:] = [-1, 3, 3]
    assert L.ctuppm_fab_elems(ctypes.byref(b), 0, ctypes.byref(e)) == ctuppm.EINVAL
    assert L.ctuppm_num_stages() == len(ctuppm.stage_names())


def test_no_cpu_fallback_without_gpu():
    import torch
    from paper_1711_06203_amd import ctuppm
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(ctuppm.CtuError):
        ctuppm.Context()
