"""Plain FP64 CPU oracle of the unsplit CTU/PPM advance (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It loads ``liboracle.so``, compiled from
``ctu_oracle.c`` (plain C, gcc -O2 -fopenmp -ffp-contract=off), which shares
no code with the HIP path.  The two-level step of the method (coarse
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


MAXSPEC = 16


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("small_dens", ctypes.c_double), ("small_pres", ctypes.c_double),
                ("grav_z", ctypes.c_double), ("dx", ctypes.c_double * 3),
                ("bc_lo", ctypes.c_int * 3), ("bc_hi", ctypes.c_int * 3),
                ("inflow", ctypes.c_double * 5), ("nspec", ctypes.c_int), ("pad", ctypes.c_int),
                ("inflow_X", ctypes.c_double * MAXSPEC), ("scheme", ctypes.c_int), ("riemann", ctypes.c_int),
                ("limiter", ctypes.c_int), ("steepen", ctypes.c_int),
                ("faces_set", ctypes.c_int), ("face_lo", ctypes.c_int * 3), ("face_hi", ctypes.c_int * 3)]

SCHEMES = {"ctu": 0, "mol2": 1, "mol3": 2}


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
        L.orc_mol_stage.argtypes = [dp, dp, ip, pp, ctypes.c_double, ctypes.c_double, dp, lp]
        L.orc_mol_stage.restype = ctypes.c_int
        L.orc_twoshock.argtypes = [dp, dp, ctypes.c_int, pp, dp]
        L.orc_twoshock.restype = None
        L.orc_ppm_cell_cs.argtypes = [dp, ctypes.c_double, dp]
        L.orc_ppm_cell_cs.restype = None
        L.orc_ppm_cell_steep.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_ppm_cell_steep.restype = None
        L.orc_steep_eta.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_steep_eta.restype = ctypes.c_double
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(seq):
    return (ctypes.c_int * 3)(*[int(v) for v in seq])


def make_params(gamma, dx, cfl=0.5, bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), grav_z=0.0,
                inflow=(1.0, 0.0, 0.0, 0.0, 1.0), small_dens=1e-12, small_pres=1e-12, nspec=0,
                inflow_X=(), scheme=0, riemann=0, limiter=0, steepen=0) -> Params:
    P = Params()
    P.steepen = int(steepen)
    P.riemann = int(riemann)
    P.limiter = int(limiter)
    P.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    P.nspec = int(nspec)
    for s_, v in enumerate(inflow_X):
        P.inflow_X[s_] = v
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
    P = make_params(prob.gamma, dx, prob.cfl, prob.bc_lo, prob.bc_hi, prob.grav_z, prob.inflow,
                    prob.small_dens, prob.small_pres, getattr(prob, "nspec", 0), getattr(prob, "inflow_X", ()),
                    getattr(prob, "scheme", 0), getattr(prob, "riemann", 0), getattr(prob, "limiter", 0),
                    getattr(prob, "steepen", 0))
    if fine:  # the fine rectangle lies inside the domain: none of its faces is a wall
        return with_faces(P, (_FAR,) * 3, (_FAR,) * 3)
    return P


_FAR = -(1 << 30)


def with_faces(P: Params, face_lo, face_hi) -> Params:
    """A copy of P for a box whose domain boundaries lie at the box-local face
    indices face_lo, face_hi (reflecting walls are imposed there)."""
    Q = Params()
    ctypes.memmove(ctypes.byref(Q), ctypes.byref(P), ctypes.sizeof(Params))
    Q.faces_set = 1
    for d in range(3):
        Q.face_lo[d] = int(face_lo[d])
        Q.face_hi[d] = int(face_hi[d])
    return Q


def grow(Uvalid: np.ndarray, fill=np.nan) -> np.ndarray:
    """Whole-domain valid state (5, nz, ny, nx) -> grown array with ghost cells."""
    nz, ny, nx = Uvalid.shape[1:]
    G = np.full((Uvalid.shape[0], nz + 2 * NG, ny + 2 * NG, nx + 2 * NG), fill)
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
    nv = G.shape[0]
    if nv != 5 + P.nspec:
        raise ValueError("state components do not match nspec")
    if stages:
        hs = (nz + 2, ny + 2, nx + 2)
        st = Stages()
        arrays["q"] = np.full((nv + 1,) + G.shape[1:], np.nan)
        arrays["phi"] = np.full((1,) + hs, np.nan)
        st.q = _dp(arrays["q"])
        st.phi = _dp(arrays["phi"])
        for d in range(3):
            for key in ("ql", "qr", "fn", "ff"):
                arrays[f"{key}{d}"] = np.full((nv,) + hs, np.nan)
                getattr(st, key)[d] = _dp(arrays[f"{key}{d}"])
        for p in range(6):
            arrays[f"f1{p}"] = np.full((nv,) + hs, np.nan)
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


def twoshock(L: Sequence[float], R: Sequence[float], d: int, gamma: float, small_dens: float = 1e-12,
             small_pres: float = 1e-12) -> np.ndarray:
    """Two-shock Riemann flux of permuted primitive states (rho, u_n, u_t1, u_t2, p),
    returned in global conserved order for a sweep along d."""
    P = make_params(gamma, (1.0, 1.0, 1.0), small_dens=small_dens, small_pres=small_pres)
    l = np.ascontiguousarray(L, dtype=np.float64)
    r = np.ascontiguousarray(R, dtype=np.float64)
    F = np.zeros(5)
    lib().orc_twoshock(_dp(l), _dp(r), int(d), ctypes.byref(P), _dp(F))
    return F


def hllc(L: Sequence[float], R: Sequence[float], d: int, gamma: float) -> np.ndarray:
    P = make_params(gamma, (1.0, 1.0, 1.0))
    l = np.ascontiguousarray(L, dtype=np.float64)
    r = np.ascontiguousarray(R, dtype=np.float64)
    F = np.zeros(5)
    lib().orc_hllc(_dp(l), _dp(r), int(d), ctypes.byref(P), _dp(F))
    return F


def ppm_cell(a: Sequence[float], phi: float = 1.0, limiter: int = 0, eta: float = 0.0) -> np.ndarray:
    """(aL, aR, da, a6) of the middle cell of a five-cell stencil (limiter 0:
    CW84, 1: Colella & Sekora 2008; eta: CW84 contact steepening weight)."""
    arr = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros(4)
    if limiter == 1:
        lib().orc_ppm_cell_cs(_dp(arr), float(phi), _dp(out))
    else:
        lib().orc_ppm_cell_steep(_dp(arr), float(phi), float(eta), _dp(out))
    return out


def steep_eta(r: Sequence[float], pm: float, pp: float, gamma: float) -> float:
    """CW84 contact-steepening weight of the middle cell of a density stencil."""
    arr = np.ascontiguousarray(r, dtype=np.float64)
    return float(lib().orc_steep_eta(_dp(arr), float(pm), float(pp), float(gamma)))


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
    G = Ufull_grown_filled
    if P.scheme != 0:
        raise ValueError("MOL schemes: use sample_step_mol on a periodic domain")
    N = [G.shape[3] - 2 * NG, G.shape[2] - 2 * NG, G.shape[1] - 2 * NG]
    out = np.zeros((len(cells), G.shape[0]))
    for s, (i, j, k) in enumerate(cells):
        loc = np.ascontiguousarray(G[:, k:k + 2 * NG + 1, j:j + 2 * NG + 1, i:i + 2 * NG + 1])
        c = (i, j, k)  # the one-cell box is domain cell c: the domain's faces sit at -c and N - c
        Pc = with_faces(P, [-c[d] for d in range(3)], [N[d] - c[d] for d in range(3)])
        Gn, _ = advance_box(loc, Pc, dt)
        out[s] = Gn[:, NG, NG, NG]
    return out


def mol_stage(Gs: np.ndarray, P: Params, dt: float, G0: Optional[np.ndarray] = None,
              c: float = 0.0) -> Tuple[np.ndarray, np.ndarray]:
    """One MOL Runge-Kutta stage on a grown array with filled ghosts: valid cells
    of the result are T = Us + dt L(Us), or U0 + c (T - U0) when G0 is given;
    ghosts are copied from Gs.  Returns (result, counters)."""
    Gs = np.ascontiguousarray(Gs, dtype=np.float64)
    n = _ip([Gs.shape[3] - 2 * NG, Gs.shape[2] - 2 * NG, Gs.shape[1] - 2 * NG])
    out = Gs.copy()
    cnt = np.zeros(NCNT, dtype=np.int64)
    g0 = None if G0 is None else np.ascontiguousarray(G0, dtype=np.float64)
    rc = lib().orc_mol_stage(_dp(Gs), _dp(g0) if g0 is not None else None, n, ctypes.byref(P), float(dt),
                             float(c), _dp(out), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
    if rc:
        raise RuntimeError(f"orc_mol_stage failed ({rc})")
    return out, cnt


def sample_step_mol(Uvalid: np.ndarray, P: Params, dt: float, cells: Sequence[Tuple[int, int, int]]) -> np.ndarray:
    """U^{n+1} of the MOL-RK2 step at chosen cells of a periodic domain, each on
    its own: stage 1 over the 9^3 cells around the sample (from their 17^3
    periodic neighbourhood), then stage 2 on the sample cell from the 9^3
    neighbourhood of the stage-1 state."""
    if P.scheme != 1:
        raise ValueError("sampled MOL steps are written for SSP-RK2")
    R = 2 * NG
    nz, ny, nx = Uvalid.shape[1:]
    out = np.zeros((len(cells), Uvalid.shape[0]))
    for s, (i, j, k) in enumerate(cells):
        iz = np.arange(k - R, k + R + 1) % nz
        iy = np.arange(j - R, j + R + 1) % ny
        ix = np.arange(i - R, i + R + 1) % nx
        loc = np.ascontiguousarray(Uvalid[:, iz][:, :, iy][:, :, :, ix])
        W1, _ = mol_stage(loc, P, dt)
        core = (slice(None), slice(NG, NG + 2 * NG + 1), slice(NG, NG + 2 * NG + 1), slice(NG, NG + 2 * NG + 1))
        Un, _ = mol_stage(np.ascontiguousarray(W1[core]), P, dt, np.ascontiguousarray(loc[core]), 0.5)
        out[s] = Un[:, NG, NG, NG]
    return out


# ----------------------------------------------------------------------------
# two levels: coarse whole domain + one fine rectangular patch (ratio 2)
# ----------------------------------------------------------------------------
#
# The paper's integration on a grid hierarchy (section 3.2) advances the coarse
# level, advances the fine level in two half steps to the same time, then
# synchronises the levels.  The synchronisation follows Berger & Colella
# (1989): the coarse fluxes at the coarse-fine faces are replaced by the time-
# and area-averaged fine fluxes (a flux register added back to the neighbouring
# uncovered coarse cells), and covered coarse cells take the average of their
# eight fine children.  Fine ghost cells come from the coarse state,
# interpolated linearly in time and with MC-limited slopes in space.


def _mc_slope(am, a0, ap):
    """Monotonised-central slope, elementwise, in the same operation order as
    the box advance's (CW84 eq. 1.7-1.8)."""
    dm = a0 - am
    dp = ap - a0
    dc = 0.5 * (ap - am)
    lim = np.minimum(np.abs(dc), np.minimum(2.0 * np.abs(dm), 2.0 * np.abs(dp)))
    return np.where(dm * dp > 0.0, np.copysign(lim, dc), 0.0)


def cf_interp(Uc_region: np.ndarray, region_lo, fine_cells) -> np.ndarray:
    """Conservative MC-linear interpolation of fine cells from a coarse region.

    Uc_region[:, k, j, i] holds coarse cell region_lo + (i, j, k).  fine_cells is
    an (N, 3) array of global fine indices (I, J, K); each takes its coarse
    parent's value plus s_x d_x + s_y d_y + s_z d_z (summed in that order),
    s = -1/4 for an even fine index, +1/4 for an odd one."""
    fc = np.asarray(fine_cells, dtype=np.int64)
    par = fc // 2
    loc = par - np.asarray(region_lo, dtype=np.int64)
    out = np.empty((Uc_region.shape[0], len(fc)))
    for m in range(Uc_region.shape[0]):
        A = Uc_region[m]
        c = A[loc[:, 2], loc[:, 1], loc[:, 0]]
        val = c.copy()
        for d in range(3):
            e = np.zeros(3, dtype=np.int64)
            e[d] = 1
            lm = loc - e
            lp = loc + e
            sl = _mc_slope(A[lm[:, 2], lm[:, 1], lm[:, 0]], c, A[lp[:, 2], lp[:, 1], lp[:, 0]])
            s = np.where(fc[:, d] % 2 == 0, -0.25, 0.25)
            val = val + s * sl
        out[m] = val
    return out


def fine_ghost_values(Rn: np.ndarray, Rn1: np.ndarray, theta: float, region_lo, fine_cells) -> np.ndarray:
    """Fine ghost values at substep time t^n + theta dt_c: the coarse state
    interpolated linearly in time, (1 - theta) U^n + theta U^{n+1}, then
    conservatively in space (cf_interp)."""
    Ut = (1.0 - theta) * Rn + theta * Rn1
    return cf_interp(Ut, region_lo, fine_cells)


def _face_sl(d, lo, hi, idx):
    """Slice of halo-1 face array axis order [m, k, j, i] for faces `idx` along d
    and cells [lo, hi] (inclusive, box-local) across."""
    sl = [slice(None)] * 4
    for e in range(3):
        ax = 3 - e
        if e == d:
            sl[ax] = slice(idx + 1, idx + 2)
        else:
            sl[ax] = slice(lo[e] + 1, hi[e] + 2)
    return tuple(sl)


def two_level_step(Gc: np.ndarray, Gf: np.ndarray, clo, chi, Pc: Params, Pf: Params):
    """One coarse step of the two-level method with one fine patch.

    Gc: whole-domain coarse grown array; Gf: grown array of the fine patch,
    which covers coarse cells clo..chi (inclusive), i.e. fine cells
    2 clo .. 2 chi + 1.  The patch must lie at least 3 coarse cells inside the
    domain.  Returns (Gc, Gf, dt_c, counters); the arrays are updated copies."""
    Gc_new, Gfs, dt_c, cnt = two_level_step_patches(Gc, [(Gf, clo, chi)], Pc, Pf)
    return Gc_new, Gfs[0], dt_c, cnt


def two_level_step_patches(Gc: np.ndarray, patches, Pc: Params, Pf: Params):
    """One coarse step of the two-level method (section 3.2) with a fine level
    made of several rectangular patches (section 3, figure 1).

    patches: list of (Gf, clo, chi), Gf the grown array of a patch covering
    coarse cells clo..chi (inclusive); the patches are disjoint and lie at
    least 3 coarse cells inside the domain.  A fine ghost cell inside another
    patch takes that patch's value at the same time; the others are
    interpolated from the coarse level.  The flux register holds the coarse
    faces between a patch and an uncovered coarse cell only.  Returns (Gc,
    [Gf], dt_c, counters) with updated copies."""
    P = []
    for Gf, clo, chi in patches:
        clo = np.asarray(clo, dtype=np.int64)
        chi = np.asarray(chi, dtype=np.int64)
        P.append({"G": np.array(Gf, dtype=np.float64, copy=True), "clo": clo, "chi": chi,
                  "flo": 2 * clo, "nf": 2 * (chi - clo + 1)})
    Gc = np.array(Gc, dtype=np.float64, copy=True)
    fill_domain(Gc, Pc)
    s_c = signal_speed(Gc, Pc)
    s_f = max(signal_speed(p["G"], Pf) for p in P)
    a = Pc.cfl / s_c
    b = 2.0 * (Pc.cfl / s_f)
    dt_c = a if a < b else b
    dt_f = 0.5 * dt_c
    cnt = np.zeros(NCNT, dtype=np.int64)
    Uc_old = Gc.copy()
    Gc_new, c1, st = advance_box(Gc, Pc, dt_c, stages=True)
    cnt += c1
    # coarse cells under some patch
    ncz, ncy, ncx = (Gc.shape[1] - 2 * NG, Gc.shape[2] - 2 * NG, Gc.shape[3] - 2 * NG)
    covered = np.zeros((ncz, ncy, ncx), dtype=bool)
    for p in P:
        covered[p["clo"][2]:p["chi"][2] + 1, p["clo"][1]:p["chi"][1] + 1, p["clo"][0]:p["chi"][0] + 1] = True
    # flux register on the patch faces: the coarse flux dt_c F_c now, the fine
    # sum S = sum over substeps of the four sub-face fluxes dt_f F_f (summed as
    # a pairwise tree), and R = dt_c F_c - S / 4 at reflux time; `mask` marks
    # the faces whose outside coarse cell no patch covers
    for p in P:
        clo, chi = p["clo"], p["chi"]
        p["Fc"], p["S"], p["mask"] = {}, {}, {}
        for d in range(3):
            for side, face in ((0, int(clo[d])), (1, int(chi[d]) + 1)):
                p["Fc"][(d, side)] = dt_c * st[f"ff{d}"][_face_sl(d, clo, chi, face)]
                p["S"][(d, side)] = np.zeros_like(p["Fc"][(d, side)])
                out = int(clo[d]) - 1 if side == 0 else int(chi[d]) + 1
                sl = [None] * 3
                for e in range(3):
                    sl[2 - e] = slice(out, out + 1) if e == d else slice(int(clo[e]), int(chi[e]) + 1)
                p["mask"][(d, side)] = ~covered[tuple(sl)][None]
    # coarse region for interpolation: the patches' bounding box grown by 3 coarse cells
    rlo = np.min([p["clo"] for p in P], axis=0) - 3
    rhi = np.max([p["chi"] for p in P], axis=0) + 3

    def region(G):
        return G[:, NG + rlo[2]:NG + rhi[2] + 1, NG + rlo[1]:NG + rhi[1] + 1, NG + rlo[0]:NG + rhi[0] + 1]
    Rn, Rn1 = region(Uc_old), region(Gc_new)
    # ghost cells of every patch (box-local and global fine indices), in
    # grown-array order, and the patch (if any) whose valid cells hold each
    for p in P:
        nf = p["nf"]
        gz, gy, gx = np.meshgrid(np.arange(-NG, nf[2] + NG), np.arange(-NG, nf[1] + NG),
                                 np.arange(-NG, nf[0] + NG), indexing="ij")
        ghost = ~((gx >= 0) & (gx < nf[0]) & (gy >= 0) & (gy < nf[1]) & (gz >= 0) & (gz < nf[2]))
        p["gloc"] = np.stack([gx[ghost], gy[ghost], gz[ghost]], axis=1)
        glob = p["gloc"] + p["flo"]
        src = np.full(len(glob), -1, dtype=np.int64)
        for q, o in enumerate(P):
            inside = np.all((glob >= o["flo"]) & (glob < o["flo"] + o["nf"]), axis=1)
            src[inside] = q
        p["gsrc"] = src
    for sub, theta in enumerate((0.0, 0.5)):
        # every patch's ghosts first (from the other patches' current valid
        # cells, else from the coarse level), then every patch's advance
        for p in P:
            loc, src = p["gloc"], p["gsrc"]
            glob = loc + p["flo"]
            interp = src < 0
            vals = fine_ghost_values(Rn, Rn1, theta, rlo, glob[interp])
            G = p["G"]
            for m in range(G.shape[0]):
                G[m][loc[interp, 2] + NG, loc[interp, 1] + NG, loc[interp, 0] + NG] = vals[m]
            for q, o in enumerate(P):
                sel = src == q
                if not sel.any():
                    continue
                ol = glob[sel] - o["flo"]
                for m in range(G.shape[0]):
                    G[m][loc[sel, 2] + NG, loc[sel, 1] + NG, loc[sel, 0] + NG] = \
                        o["G"][m][ol[:, 2] + NG, ol[:, 1] + NG, ol[:, 0] + NG]
        new = []
        for p in P:
            Gf_new, c2, stf = advance_box(p["G"], Pf, dt_f, stages=True)
            cnt += c2
            nf = p["nf"]
            # register: add the four fine sub-faces of each coarse face as
            # ((t00 + t10) + (t01 + t11)), t = dt_f F_f, first transverse index fastest
            for d in range(3):
                t1, t2 = [e for e in range(3) if e != d]
                for side, face in ((0, 0), (1, int(nf[d]))):
                    sl = [slice(None)] * 4
                    for e in range(3):
                        sl[3 - e] = slice(face + 1, face + 2) if e == d else slice(1, nf[e] + 1)
                    Fd = stf[f"ff{d}"][tuple(sl)]

                    def sub_face(q1, q2):
                        sl2 = [slice(None)] * 4
                        for e in range(3):
                            if e != d:
                                sl2[3 - e] = slice(q1 if e == t1 else q2, None, 2)
                        return dt_f * Fd[tuple(sl2)]
                    p["S"][(d, side)] = p["S"][(d, side)] + ((sub_face(0, 0) + sub_face(1, 0))
                                                             + (sub_face(0, 1) + sub_face(1, 1)))
            new.append(Gf_new)
        for p, G in zip(P, new):
            p["G"] = G
    # average down onto covered coarse cells: 1/8 of the eight children summed
    # as a pairwise tree ((000 + 100) + (010 + 110)) + ((001 + 101) + (011 + 111))
    for p in P:
        nf, clo, chi = p["nf"], p["clo"], p["chi"]
        fv = p["G"][:, NG:NG + nf[2], NG:NG + nf[1], NG:NG + nf[0]]
        ch = lambda i, j, k: fv[:, k::2, j::2, i::2]
        avg = 0.125 * (((ch(0, 0, 0) + ch(1, 0, 0)) + (ch(0, 1, 0) + ch(1, 1, 0)))
                       + ((ch(0, 0, 1) + ch(1, 0, 1)) + (ch(0, 1, 1) + ch(1, 1, 1))))
        Gc_new[:, NG + clo[2]:NG + chi[2] + 1, NG + clo[1]:NG + chi[1] + 1, NG + clo[0]:NG + chi[0] + 1] = avg
    # reflux the uncovered neighbours of the patch faces: x then y then z, the
    # low side of the fine level before the high side, so a coarse cell beside
    # the fine level on several sides takes its corrections in that order
    for d in range(3):
        rdx = 1.0 / Pc.dx[d]
        for side in (0, 1):
            for p in P:
                clo, chi = p["clo"], p["chi"]
                cell = int(clo[d]) - 1 if side == 0 else int(chi[d]) + 1
                sl = [slice(None)] * 4
                for e in range(3):
                    sl[3 - e] = slice(NG + cell, NG + cell + 1) if e == d else slice(NG + clo[e], NG + chi[e] + 1)
                R = p["Fc"][(d, side)] - 0.25 * p["S"][(d, side)]
                cur = Gc_new[tuple(sl)]
                upd = cur + R * rdx if side == 0 else cur - R * rdx
                Gc_new[tuple(sl)] = np.where(p["mask"][(d, side)], upd, cur)
    return Gc_new, [p["G"] for p in P], dt_c, cnt


def tag_cells(Uvalid: np.ndarray, P: Params, threshold: float) -> np.ndarray:
    """Refinement tags (nz, ny, nx): a cell is tagged when, along some
    direction, |rho(+1) - rho(-1)| > threshold (rho(+1) + rho(-1)), with the
    domain's ghost cells filled."""
    G = fill_domain(grow(np.asarray(Uvalid, dtype=np.float64)), P)
    rho = G[0]
    nz, ny, nx = Uvalid.shape[1:]
    core = (slice(NG, NG + nz), slice(NG, NG + ny), slice(NG, NG + nx))
    tags = np.zeros((nz, ny, nx), dtype=bool)
    for axis in range(3):  # array axes z, y, x
        hi = list(core)
        lo = list(core)
        hi[axis] = slice(core[axis].start + 1, core[axis].stop + 1)
        lo[axis] = slice(core[axis].start - 1, core[axis].stop - 1)
        rp, rm = rho[tuple(hi)], rho[tuple(lo)]
        tags |= np.abs(rp - rm) > threshold * (rp + rm)
    return tags


def regrid_fine(Uc: np.ndarray, Uf_old: np.ndarray, old_lo, new_lo, new_n) -> np.ndarray:
    """New fine-level state (valid cells of the new rectangle, fine index
    new_lo, extent new_n = (nx, ny, nz)): cells inside the old fine rectangle
    (fine index old_lo, array Uf_old) keep their old values, the others are
    interpolated from the coarse valid state Uc (cf_interp; the patch lies at
    least 3 coarse cells inside the domain)."""
    new_lo = np.asarray(new_lo)
    nx, ny, nz = new_n
    gz, gy, gx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    fidx = np.stack([gx.ravel() + new_lo[0], gy.ravel() + new_lo[1], gz.ravel() + new_lo[2]], axis=1)
    vals = cf_interp(Uc, (0, 0, 0), fidx).reshape((Uc.shape[0], nz, ny, nx))
    olo = np.asarray(old_lo)
    on = np.asarray(Uf_old.shape[1:][::-1])
    lo = np.maximum(olo, new_lo)
    hi = np.minimum(olo + on, new_lo + np.asarray(new_n))
    if np.all(hi > lo):
        dst = (slice(None),) + tuple(slice(lo[d] - new_lo[d], hi[d] - new_lo[d]) for d in (2, 1, 0))
        src = (slice(None),) + tuple(slice(lo[d] - olo[d], hi[d] - olo[d]) for d in (2, 1, 0))
        vals[dst] = Uf_old[src]
    return vals


def regrid_patches(Uc: np.ndarray, old, new):
    """New fine patches (fine index lo, extent (nx, ny, nz)) of a regrid: cells
    under an old patch (list of (fine index lo, valid state)) keep its values,
    the others are interpolated from the coarse valid state Uc (cf_interp).
    Returns one array per new patch."""
    out = []
    for lo, n in new:
        lo = np.asarray(lo)
        nx, ny, nz = n
        gz, gy, gx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        fidx = np.stack([gx.ravel() + lo[0], gy.ravel() + lo[1], gz.ravel() + lo[2]], axis=1)
        vals = cf_interp(Uc, (0, 0, 0), fidx).reshape((Uc.shape[0], nz, ny, nx))
        for olo, U in old:
            olo = np.asarray(olo)
            on = np.asarray(U.shape[1:][::-1])
            a = np.maximum(olo, lo)
            b = np.minimum(olo + on, lo + np.asarray(n))
            if np.all(b > a):
                dst = (slice(None),) + tuple(slice(a[d] - lo[d], b[d] - lo[d]) for d in (2, 1, 0))
                src = (slice(None),) + tuple(slice(a[d] - olo[d], b[d] - olo[d]) for d in (2, 1, 0))
                vals[dst] = U[src]
        out.append(vals)
    return out


def fine_patches(prob):
    """The fine patches of a two-level problem as (fine index lo, valid state)."""
    pat = getattr(prob, "fine_patches", None)
    if pat:
        return [(tuple(int(v) for v in lo), np.asarray(U)) for lo, U in pat]
    return [(tuple(int(v) for v in prob.fine_lo), np.asarray(prob.U0_fine))]


def run_two_level_from(prob, Uc: np.ndarray, Uf: np.ndarray, fine_lo, nsteps: int):
    """run_two_level from given coarse and fine states (fine rectangle at fine_lo)."""
    import dataclasses
    p2 = dataclasses.replace(prob, U0=Uc, U0_fine=Uf, fine_lo=tuple(int(v) for v in fine_lo), fine_patches=None)
    return run_two_level(p2, nsteps)


def run_two_level(prob, nsteps: int):
    """Two-level run of a workloads.Problem with fine patches (fine_patches, or
    the one rectangle U0_fine at fine_lo).  Returns (coarse valid, fine valid,
    dts, counters); the fine valid state is one array for one patch, a list of
    arrays (in patch order) for several."""
    Pc = params_of(prob)
    Pf = params_of(prob, fine=True)
    Gc = grow(prob.U0)
    pats = []
    for flo, U in fine_patches(prob):
        flo = np.array(flo)
        nf = np.array(U.shape[1:][::-1])
        pats.append([grow(U), flo // 2, (flo + nf) // 2 - 1])
    dts = []
    cnt = np.zeros(NCNT, dtype=np.int64)
    for _ in range(nsteps):
        Gc, Gfs, dt, c = two_level_step_patches(Gc, pats, Pc, Pf)
        for p, G in zip(pats, Gfs):
            p[0] = G
        dts.append(dt)
        cnt += c
    fine = [valid(p[0]) for p in pats]
    return valid(Gc), (fine[0] if len(fine) == 1 else fine), np.array(dts), cnt
