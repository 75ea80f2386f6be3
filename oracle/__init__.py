"""Plain FP64 CPU oracle of the unsplit CTU/PPM advance (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It loads ``liboracle.so``, compiled from
``ctu_oracle.c`` (plain C, gcc -O2 -fopenmp -ffp-contract=off), which shares
no code with the HIP path.  The two-level driver of the method (coarse
advance, two fine substeps, average down, reflux; section 3.2) is written here
in numpy on top of the C box advance.

Parity unpinned parts: the paper gives only "unsplit piecewise parabolic
method" (section 3.2), so the scheme's details are the published methods it
names (cited in ctu_oracle.c); they are pinned by exact solutions, invariants
and convergence in tests/test_oracle_pins.py, not by numbers from the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ctu_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NG = 4
NCNT = 5
BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_INFLOW = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle library in place."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("small_dens", ctypes.c_double), ("small_pres", ctypes.c_double),
                ("grav_z", ctypes.c_double), ("dx", ctypes.c_double * 3),
                ("bc_lo", ctypes.c_int * 3), ("bc_hi", ctypes.c_int * 3),
                ("inflow", ctypes.c_double * 5)]


class Stages(ctypes.Structure):
    _P = ctypes.POINTER(ctypes.c_double)
    _fields_ = [("q", _P), ("phi", _P), ("ql", _P * 3), ("qr", _P * 3), ("fn", _P * 3),
                ("f1", _P * 6), ("ff", _P * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_longlong)
        pp = ctypes.POINTER(Params)
        L.orc_advance_box.argtypes = [dp, ip, pp, ctypes.c_double, dp, lp, ctypes.POINTER(Stages)]
        L.orc_advance_box.restype = ctypes.c_int
        L.orc_fill_domain.argtypes = [dp, ip, pp]
        L.orc_fill_domain.restype = None
        L.orc_signal_speed.argtypes = [dp, ip, pp]
        L.orc_signal_speed.restype = ctypes.c_double
        L.orc_step.argtypes = [dp, ip, pp, ctypes.c_double, dp, lp]
        L.orc_step.restype = ctypes.c_int
        L.orc_run.argtypes = [dp, ip, pp, ctypes.c_int, ctypes.c_double, dp, lp]
        L.orc_run.restype = ctypes.c_int
        L.orc_hllc.argtypes = [dp, dp, ctypes.c_int, pp, dp]
        L.orc_hllc.restype = None
        L.orc_ppm_cell.argtypes = [dp, ctypes.c_double, dp]
        L.orc_ppm_cell.restype = None
        L.orc_iplus.argtypes = [ctypes.c_double] * 4
        L.orc_iplus.restype = ctypes.c_double
        L.orc_iminus.argtypes = [ctypes.c_double] * 4
        L.orc_iminus.restype = ctypes.c_double
        L.orc_trace_cell.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, dp, dp]
        L.orc_trace_cell.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(seq):
    return (ctypes.c_int * 3)(*[int(v) for v in seq])


def make_params(gamma, dx, cfl=0.5, bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), grav_z=0.0,
                inflow=(1.0, 0.0, 0.0, 0.0, 1.0), small_dens=1e-12, small_pres=1e-12) -> Params:
    P = Params()
    P.gamma, P.cfl, P.small_dens, P.small_pres, P.grav_z = gamma, cfl, small_dens, small_pres, grav_z
    for d in range(3):
        P.dx[d] = dx[d]
        P.bc_lo[d] = bc_lo[d]
        P.bc_hi[d] = bc_hi[d]
    for m in range(5):
        P.inflow[m] = inflow[m]
    return P


def params_of(prob, fine: bool = False) -> Params:
    dx = prob.dx
    if fine:
        dx = tuple(v / 2.0 for v in dx)
    return make_params(prob.gamma, dx, prob.cfl, prob.bc_lo, prob.bc_hi, prob.grav_z, prob.inflow,
                       prob.small_dens, prob.small_pres)


def grow(Uvalid: np.ndarray, fill=np.nan) -> np.ndarray:
    """Whole-domain valid state (5, nz, ny, nx) -> grown array with ghost cells."""
    nz, ny, nx = Uvalid.shape[1:]
    G = np.full((5, nz + 2 * NG, ny + 2 * NG, nx + 2 * NG), fill)
    G[:, NG:NG + nz, NG:NG + ny, NG:NG + nx] = Uvalid
    return G


def valid(G: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(G[:, NG:-NG, NG:-NG, NG:-NG])


def fill_domain(G: np.ndarray, P: Params) -> np.ndarray:
    n = (G.shape[3] - 2 * NG, G.shape[2] - 2 * NG, G.shape[1] - 2 * NG)
    lib().orc_fill_domain(_dp(G), _ip(n), ctypes.byref(P))
    return G


def signal_speed(G: np.ndarray, P: Params) -> float:
    n = (G.shape[3] - 2 * NG, G.shape[2] - 2 * NG, G.shape[1] - 2 * NG)
    return lib().orc_signal_speed(_dp(G), _ip(n), ctypes.byref(P))


def advance_box(G: np.ndarray, P: Params, dt: float, stages: bool = False):
    """Advance a grown box whose ghosts are filled; returns (Gnew, counters[, stages])."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    nz, ny, nx = (G.shape[1] - 2 * NG, G.shape[2] - 2 * NG, G.shape[3] - 2 * NG)
    n = (nx, ny, nz)
    Gn = G.copy()
    cnt = (ctypes.c_longlong * NCNT)()
    st = None
    arrays: Dict[str, np.ndarray] = {}
    if stages:
        hs = (nz + 2, ny + 2, nx + 2)
        st = Stages()
        arrays["q"] = np.full((6,) + G.shape[1:], np.nan)
        arrays["phi"] = np.full((1,) + hs, np.nan)
        st.q = _dp(arrays["q"])
        st.phi = _dp(arrays["phi"])
        for d in range(3):
            for key in ("ql", "qr", "fn", "ff"):
                arrays[f"{key}{d}"] = np.full((5,) + hs, np.nan)
                getattr(st, key)[d] = _dp(arrays[f"{key}{d}"])
        for p in range(6):
            arrays[f"f1{p}"] = np.full((5,) + hs, np.nan)
            st.f1[p] = _dp(arrays[f"f1{p}"])
    rc = lib().orc_advance_box(_dp(G), _ip(n), ctypes.byref(P), float(dt), _dp(Gn), cnt,
                               ctypes.byref(st) if st is not None else None)
    if rc:
        raise RuntimeError(f"orc_advance_box failed: {rc}")
    if stages:
        return Gn, np.array(cnt[:]), arrays
    return Gn, np.array(cnt[:])


def run(Uvalid: np.ndarray, P: Params, nsteps: int, dt_fixed: Optional[float] = None):
    """Single-level run on a whole domain: returns (U valid, dts, counters)."""
    G = grow(np.asarray(Uvalid, dtype=np.float64))
    nz, ny, nx = Uvalid.shape[1:]
    dts = np.zeros(max(nsteps, 1))
    cnt = (ctypes.c_longlong * NCNT)()
    rc = lib().orc_run(_dp(G), _ip((nx, ny, nz)), ctypes.byref(P), int(nsteps),
                       float(dt_fixed) if dt_fixed else 0.0, _dp(dts), cnt)
    if rc:
        raise RuntimeError(f"orc_run failed: {rc}")
    return valid(G), dts[:nsteps], np.array(cnt[:])


def run_problem(prob, nsteps: Optional[int] = None, dt_fixed: Optional[float] = None):
    return run(prob.U0, params_of(prob), prob.steps if nsteps is None else nsteps, dt_fixed)


def hllc(L: Sequence[float], R: Sequence[float], d: int, gamma: float) -> np.ndarray:
    P = make_params(gamma, (1.0, 1.0, 1.0))
    l = np.ascontiguousarray(L, dtype=np.float64)
    r = np.ascontiguousarray(R, dtype=np.float64)
    F = np.zeros(5)
    lib().orc_hllc(_dp(l), _dp(r), int(d), ctypes.byref(P), _dp(F))
    return F


def ppm_cell(a: Sequence[float], phi: float = 1.0) -> np.ndarray:
    """(aL, aR, da, a6) of the middle cell of a five-cell stencil."""
    arr = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros(4)
    lib().orc_ppm_cell(_dp(arr), float(phi), _dp(out))
    return out


def iplus(aR, da, a6, sig) -> float:
    return lib().orc_iplus(aR, da, a6, sig)


def iminus(aL, da, a6, sig) -> float:
    return lib().orc_iminus(aL, da, a6, sig)


def trace_cell(par: np.ndarray, rho: float, un: float, c: float, dtdx: float):
    par = np.ascontiguousarray(par, dtype=np.float64).reshape(5, 4)
    qL = np.zeros(5)
    qR = np.zeros(5)
    lib().orc_trace_cell(_dp(par), rho, un, c, dtdx, _dp(qL), _dp(qR))
    return qL, qR


def sample_step(Ufull_grown_filled: np.ndarray, P: Params, dt: float,
                cells: Sequence[Tuple[int, int, int]]) -> np.ndarray:
    """U^{n+1} at chosen cells (i, j, k), each computed on its own from the 9^3
    neighbourhood of a whole-domain grown array whose ghosts are filled."""
    out = np.zeros((len(cells), 5))
    G = Ufull_grown_filled
    for s, (i, j, k) in enumerate(cells):
        loc = np.ascontiguousarray(G[:, k:k + 2 * NG + 1, j:j + 2 * NG + 1, i:i + 2 * NG + 1])
        Gn, _ = advance_box(loc, P, dt)
        out[s] = Gn[:, NG, NG, NG]
    return out
