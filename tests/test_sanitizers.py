"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the C oracle and the library's host-side clustering are rebuilt with gcc /
g++ and the sanitizers, then driven through a child Python process (the
sanitizer runtime preloaded) over small problems of every scheme, solver and
limiter, two levels, and random tag fields.  Any report fails the test."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not out or not os.path.isabs(out) or not os.path.exists(out):
        pytest.skip("no AddressSanitizer runtime for gcc here")
    return out


def _child(script, preload):
    env = dict(os.environ)
    env.update(LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2",
               PYTHONPATH=ROOT + os.pathsep + os.path.join(ROOT, "tests"))
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env, timeout=600)
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-4000:]
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    pre = _runtime()
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", *SAN, "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", lib,
                           os.path.join(ROOT, "oracle", "ctu_oracle.c"), "-lm"])
    script = textwrap.dedent(f"""
        import numpy as np
        import oracle
        oracle._LIB = {lib!r}
        from paper_1711_06203_amd import workloads as W
        cases = []
        p = W.kelvin_helmholtz(n=(12, 10, 8), box=(12, 10, 8), nspec=2); cases.append(p)
        for var in (dict(riemann=1), dict(limiter=1), dict(steepen=1), dict(scheme=1), dict(scheme=2, riemann=1)):
            q = W.kelvin_helmholtz(n=(12, 10, 8), box=(12, 10, 8), nspec=1)
            for k, v in var.items():
                setattr(q, k, v)
            cases.append(q)
        cases.append(W.rayleigh_taylor(n=(8, 8, 16), seed=2, boxes=[((0, 0, 0), (7, 7, 15))]))
        cases.append(W.sod(n=(16, 4, 4)))
        for p in cases:
            U, dts, cnt = oracle.run_problem(p, 2)
            assert np.isfinite(U).all()
        c = W.cloud_wind(n=16, box=16, fine_box=8, fine_region=((4, 4, 4), (12, 12, 12)), nspec=1)
        rc, rf, _, _ = oracle.run_two_level(c, 1)
        assert np.isfinite(rc).all() and np.isfinite(rf).all()
        t = oracle.tag_cells(c.U0, oracle.params_of(c), 0.1)
        print("oracle ok", len(cases), int(t.sum()))
    """)
    assert "oracle ok" in _child(script, pre)


def test_clustering_under_asan_ubsan(tmp_path):
    pre = _runtime()
    lib = str(tmp_path / "libcluster_san.so")
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-fPIC", "-shared", "-I", os.path.join(ROOT, "include"),
                           "-o", lib, os.path.join(ROOT, "paper_1711_06203_amd", "csrc", "ctuppm_cluster.cpp")])
    script = textwrap.dedent(f"""
        import ctypes
        import numpy as np
        L = ctypes.CDLL({lib!r})
        class Box(ctypes.Structure):
            _fields_ = [("lo", ctypes.c_int * 3), ("hi", ctypes.c_int * 3)]
        rng = np.random.default_rng(5)
        total = 0
        for trial in range(40):
            n = rng.integers(1, 40, size=3)
            t = (rng.random((n[2], n[1], n[0])) < rng.choice([0.0, 0.01, 0.1, 0.5, 1.0])).astype(np.uint8)
            blocking = int(rng.choice([1, 2, 4, 8]))
            cap = 16 + int(np.prod([-(-int(v) // blocking) for v in n]))
            out = (Box * cap)()
            nb = ctypes.c_int()
            dims = (ctypes.c_int * 3)(*[int(v) for v in n])
            rc = L.ctuppm_cluster(t.ctypes.data_as(ctypes.c_void_p), dims, blocking, ctypes.c_double(0.7),
                                  int(rng.choice([8, 16, 64])), out, cap, ctypes.byref(nb))
            assert rc == 0, rc
            total += nb.value
        small = (Box * 1)()
        nb = ctypes.c_int()
        t = np.ones((16, 16, 16), dtype=np.uint8)
        rc = L.ctuppm_cluster(t.ctypes.data_as(ctypes.c_void_p), (ctypes.c_int * 3)(16, 16, 16), 1,
                              ctypes.c_double(0.99), 4, small, 1, ctypes.byref(nb))
        assert rc != 0  # capacity too small: an error, not an overrun
        print("cluster ok", total)
    """)
    assert "cluster ok" in _child(script, pre)
