"""Python binding of the C ABI in include/ctuppm.h (ctypes).

Argument marshalling only: PyTorch allocates the device memory (state fabs,
stage workspace) and provides the HIP stream; every step of the hydro advance
runs in the HIP kernels of ``libctuppm.so``.  There is no CPU fallback: if the
library or a GPU is missing, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctuppm.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE, ERETRY = 0, -1, -2, -3, -4, -5
FORM_PER_BOX, FORM_BATCHED, FORM_GRAPH, FORM_WAVES = 0, 1, 2, 3
FORMS = {"per_box": FORM_PER_BOX, "batched": FORM_BATCHED, "graph": FORM_GRAPH, "waves": FORM_WAVES}
SCHEME_CTU, SCHEME_MOL_RK2, SCHEME_MOL_RK3 = 0, 1, 2
SCHEMES = {"ctu": SCHEME_CTU, "mol2": SCHEME_MOL_RK2, "mol3": SCHEME_MOL_RK3}
RIEMANN_HLLC, RIEMANN_TWO_SHOCK = 0, 1
RIEMANN = {"hllc": RIEMANN_HLLC, "twoshock": RIEMANN_TWO_SHOCK}
LIMITER_CW84, LIMITER_CS = 0, 1
LIMITERS = {"cw84": LIMITER_CW84, "cs": LIMITER_CS}
NG = 4


class CtuError(RuntimeError):
    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


class Rejected(CtuError):
    """A guarded step was rejected by the retry criterion (CTUPPM_ERETRY)."""


class Box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int * 3), ("hi", ctypes.c_int * 3)]


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("small_dens", ctypes.c_double),
                ("small_pres", ctypes.c_double), ("grav_z", ctypes.c_double), ("dx", ctypes.c_double * 3),
                ("domain_lo", ctypes.c_int * 3), ("domain_hi", ctypes.c_int * 3),
                ("bc_lo", ctypes.c_int * 3), ("bc_hi", ctypes.c_int * 3), ("inflow", ctypes.c_double * 5),
                ("nspec", ctypes.c_int), ("pad", ctypes.c_int), ("inflow_X", ctypes.c_double * 16),
                ("scheme", ctypes.c_int), ("riemann", ctypes.c_int),
                ("limiter", ctypes.c_int), ("steepen", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libctuppm.so (built by paper_1711_06203_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CtuError(f"{LIB_PATH} is missing: build it with python -m paper_1711_06203_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
        llp = ctypes.POINTER(ctypes.c_longlong)
        sz = ctypes.c_size_t
        sig = {
            "ctuppm_ctx_create": [vp, ctypes.POINTER(vp)],
            "ctuppm_ctx_destroy": [vp],
            "ctuppm_problem_create": [vp, ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(ctypes.POINTER(Box)),
                                      ip, ip],
            "ctuppm_problem_destroy": [vp, ctypes.c_int],
            "ctuppm_fab_elems": [ctypes.POINTER(Box), ctypes.c_int, llp],
            "ctuppm_workspace_bytes": [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(sz)],
            "ctuppm_workspace_meta_bytes": [vp, ctypes.c_int, ctypes.POINTER(sz)],
            "ctuppm_step_guarded": [vp, ip, ctypes.c_int, ctypes.c_int],
            "ctuppm_step_static": [vp, ctypes.c_int],
            "ctuppm_set_fused": [vp, ctypes.c_int],
            "ctuppm_bandwidth_probe": [vp, ctypes.c_int, vp, vp, sz, ctypes.c_int, dp],
            "ctuppm_rejections": [vp, ctypes.c_int, llp],
            "ctuppm_rejections_seen": [vp, ctypes.c_int, llp],
            "ctuppm_bind_state": [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp)],
            "ctuppm_bind_workspace": [vp, ctypes.c_int, vp, sz],
            "ctuppm_set_fixed_dt": [vp, ctypes.c_int, ctypes.c_double],
            "ctuppm_step": [vp, ip, ctypes.c_int, ctypes.c_int],
            "ctuppm_current_state": [vp, ctypes.c_int, ip],
            "ctuppm_get_dt": [vp, ctypes.c_int, dp],
            "ctuppm_status": [vp, ctypes.c_int, llp],
            "ctuppm_set_timing": [vp, ctypes.c_int],
            "ctuppm_stage_times": [vp, dp, llp, ctypes.c_int],
            "ctuppm_num_stages": [],
            "ctuppm_stage_name": [ctypes.c_int],
            "ctuppm_stage_bytes": [vp, ctypes.c_int, ctypes.c_int, dp],
            "ctuppm_set_tuning": [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int],
            "ctuppm_set_tuning2": [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int],
            "ctuppm_set_stage_planes": [vp, ctypes.c_int, ctypes.c_int],
            "ctuppm_stage_planes": [vp, ctypes.c_int, ip, ip],
            "ctuppm_step_checked": [vp, ctypes.c_int, ctypes.c_int, ip],
            "ctuppm_set_fail_hook": [vp, ctypes.c_int, ctypes.c_int],
            "ctuppm_last_error": [vp],
            "ctuppm_tag": [vp, ctypes.c_int, ctypes.c_double, vp],
            "ctuppm_set_concurrency": [vp, ctypes.c_int],
            "ctuppm_cluster": [vp, ip, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Box), ctypes.c_int,
                               ip],
            "ctuppm_regrid": [vp, ctypes.c_int, ctypes.POINTER(Box), ctypes.c_int, ctypes.POINTER(vp),
                              ctypes.POINTER(vp)],
            "ctuppm_fill_ghosts": [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int],
            "ctuppm_compute_dt": [vp, ctypes.c_int, ctypes.c_int, vp],
            "ctuppm_advance_level": [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp],
            "ctuppm_average_down": [vp, ctypes.c_int],
            "ctuppm_reflux": [vp, ctypes.c_int],
            "ctuppm_set_wave_boxes": [vp, ctypes.c_int],
            "ctuppm_debug_stage": [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                   llp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.ctuppm_last_error.restype = ctypes.c_char_p
        L.ctuppm_stage_name.restype = ctypes.c_char_p
        _lib = L
    return _lib


EXPORTED = ["ctuppm_ctx_create", "ctuppm_ctx_destroy", "ctuppm_last_error", "ctuppm_problem_create",
            "ctuppm_problem_destroy", "ctuppm_fab_elems", "ctuppm_workspace_bytes", "ctuppm_bind_state",
            "ctuppm_bind_workspace", "ctuppm_set_fixed_dt", "ctuppm_step", "ctuppm_current_state",
            "ctuppm_get_dt", "ctuppm_status", "ctuppm_set_timing", "ctuppm_stage_times", "ctuppm_num_stages",
            "ctuppm_stage_name", "ctuppm_stage_bytes", "ctuppm_set_tuning", "ctuppm_step_checked",
            "ctuppm_set_fail_hook", "ctuppm_set_tuning2", "ctuppm_tag", "ctuppm_cluster", "ctuppm_regrid",
            "ctuppm_set_concurrency", "ctuppm_fill_ghosts", "ctuppm_compute_dt", "ctuppm_advance_level",
            "ctuppm_average_down", "ctuppm_reflux", "ctuppm_set_wave_boxes",
            "ctuppm_debug_stage", "ctuppm_workspace_meta_bytes", "ctuppm_step_guarded", "ctuppm_rejections", "ctuppm_rejections_seen",
            "ctuppm_step_static", "ctuppm_set_fused", "ctuppm_bandwidth_probe", "ctuppm_set_stage_planes",
            "ctuppm_stage_planes"]


class Context:
    """A library context on the current torch stream of the current device."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise CtuError("no GPU visible: the CTU/PPM library runs on the MI355X only")
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._side = None
        h = ctypes.c_void_p()
        self._L = lib()
        self._check(self._L.ctuppm_ctx_create(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), None)
        self.h = h

    @property
    def side_stream(self):
        """A second torch stream (default priority) for uploads beside the steps."""
        if self._side is None:
            self._side = self.torch.cuda.Stream()
        return self._side

    def _check(self, rc, h=-1):
        if rc != OK:
            msg = self._L.ctuppm_last_error(self.h if h == -1 else h)
            text = f"ctuppm error {rc}: {msg.decode() if msg else ''}"
            raise (Rejected if rc == ERETRY else CtuError)(text, rc)

    def call(self, name, *args):
        self._check(getattr(self._L, name)(self.h, *args))

    def close(self):
        if getattr(self, "h", None):
            self._L.ctuppm_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- timing
    def set_timing(self, on: bool):
        self.call("ctuppm_set_timing", int(bool(on)))

    def stage_times(self) -> Dict[str, tuple]:
        n = self._L.ctuppm_num_stages()
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_longlong * n)()
        self.call("ctuppm_stage_times", ms, cnt, n)
        return {self._L.ctuppm_stage_name(s).decode(): (ms[s], cnt[s]) for s in range(n)}

    def set_wave_boxes(self, boxes: int):
        """Boxes per wave of the waves form (they share as many scratch slots)."""
        self.call("ctuppm_set_wave_boxes", int(boxes))

    def bandwidth_probe(self, kind: str, gib: int = 2, reps: int = 10) -> float:
        """GB/s a plain streaming kernel of the library reaches: 'copy' (read +
        write), 'read' or 'write', over `gib` GiB buffers."""
        torch = self.torch
        n = (gib << 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a) if kind != "read" else a
        k = {"copy": 0, "read": 1, "write": 2}[kind]
        v = ctypes.c_double()
        self.call("ctuppm_bandwidth_probe", k, ctypes.c_void_p(a.data_ptr()),
                  ctypes.c_void_p(b.data_ptr()), n * 8, int(reps), ctypes.byref(v))
        del a, b
        return v.value

    def set_fused(self, on):
        """Cell stages: tracing (or face states) and transverse stage 1 of the
        three directions in one kernel each, the species in a stage of their
        own (True or 1, the default); 2: the same with the species inside the
        merged kernels; False or 0: one kernel per direction."""
        mode = int(on)
        if mode not in (0, 1, 2):
            raise ValueError("fused mode must be 0, 1 or 2")
        self.call("ctuppm_set_fused", mode)

    def set_concurrency(self, on: bool):
        """Graph form: run the three directions of each phase concurrently (default off)."""
        self.call("ctuppm_set_concurrency", int(bool(on)))

    def set_tuning(self, blocks_per_cu: int = 0, zseg_batched: int = 1, zseg_per_box: int = 1, ytile: int = 0):
        self.call("ctuppm_set_tuning2", int(blocks_per_cu), int(zseg_batched), int(zseg_per_box), int(ytile))

    def stage_id(self, stage) -> int:
        """Index of a stage given by name (as in stage_times) or index."""
        if isinstance(stage, int):
            return stage
        names = [self._L.ctuppm_stage_name(s).decode() for s in range(self._L.ctuppm_num_stages())]
        if stage not in names:
            raise CtuError(f"unknown stage {stage!r}", EINVAL)
        return names.index(stage)

    def set_stage_planes(self, stage, planes: int):
        """Planes per work unit of one stage (shared with the stages of its group)."""
        self.call("ctuppm_set_stage_planes", self.stage_id(stage), int(planes))

    def stage_planes(self, stage) -> Tuple[int, int]:
        """(planes per work unit, group) of a stage."""
        p, g = ctypes.c_int(), ctypes.c_int()
        self.call("ctuppm_stage_planes", self.stage_id(stage), ctypes.byref(p), ctypes.byref(g))
        return p.value, g.value

    def step(self, solvers: Sequence["Solver"], form="batched", nsteps: int = 1, guarded: bool = False):
        """Advance several problems together: one batched launch set per step
        for the problems of each (scheme, Riemann solver, limiter).  guarded:
        a problem whose new state fails keeps its old one (raises Rejected
        once the host sees a rejection)."""
        f = FORMS[form] if isinstance(form, str) else int(form)
        groups: Dict[tuple, List[int]] = {}
        for s in solvers:
            key = (scheme_id(s.prob), riemann_id(s.prob), limiter_id(s.prob), int(s.prob.steepen))
            groups.setdefault(key, []).append(s.pid)
        sets = [(ctypes.c_int * len(v))(*v) for _, v in sorted(groups.items())]
        for _ in range(nsteps):
            for pids in sets:
                self.call("ctuppm_step_guarded" if guarded else "ctuppm_step", pids, len(pids), f)


def cluster(tags: np.ndarray, blocking: int = 4, efficiency: float = 0.7, max_edge: int = 64) -> List[W.Box]:
    """Berger-Rigoutsos boxes around the tagged cells of a (nz, ny, nx) array
    (host code of the library; needs no GPU)."""
    t = np.ascontiguousarray(tags, dtype=np.uint8)
    nz, ny, nx = t.shape
    n = (ctypes.c_int * 3)(nx, ny, nz)
    b = max(1, int(blocking))
    cap = 16 + int(np.prod([-(-v // b) for v in (nx, ny, nz)]))  # boxes hold whole blocks: at most one per block
    out = (Box * cap)()
    nb = ctypes.c_int()
    rc = lib().ctuppm_cluster(t.ctypes.data_as(ctypes.c_void_p), n, int(blocking), float(efficiency), int(max_edge),
                              out, cap, ctypes.byref(nb))
    if rc != OK:
        raise CtuError(f"ctuppm_cluster failed ({rc})")
    return [(tuple(out[q].lo), tuple(out[q].hi)) for q in range(nb.value)]


def scheme_id(prob: W.Problem) -> int:
    return SCHEMES[prob.scheme] if isinstance(prob.scheme, str) else int(prob.scheme)


def riemann_id(prob: W.Problem) -> int:
    return RIEMANN[prob.riemann] if isinstance(prob.riemann, str) else int(prob.riemann)


def limiter_id(prob: W.Problem) -> int:
    return LIMITERS[prob.limiter] if isinstance(prob.limiter, str) else int(prob.limiter)


def stage_names() -> List[str]:
    L = lib()
    return [L.ctuppm_stage_name(s).decode() for s in range(L.ctuppm_num_stages())]


def _params(prob: W.Problem) -> Params:
    P = Params()
    P.gamma, P.cfl, P.small_dens, P.small_pres, P.grav_z = (prob.gamma, prob.cfl, prob.small_dens,
                                                            prob.small_pres, prob.grav_z)
    for d in range(3):
        P.dx[d] = prob.dx[d]
        P.domain_lo[d] = 0
        P.domain_hi[d] = prob.n[d] - 1
        P.bc_lo[d] = prob.bc_lo[d]
        P.bc_hi[d] = prob.bc_hi[d]
    for m in range(5):
        P.inflow[m] = prob.inflow[m]
    P.nspec = int(prob.nspec)
    P.scheme = scheme_id(prob)
    P.riemann = riemann_id(prob)
    P.limiter = limiter_id(prob)
    P.steepen = int(prob.steepen)
    for s, x in enumerate(prob.inflow_X):
        P.inflow_X[s] = x
    return P


class Solver:
    """One problem resident on the GPU: two fabs per box (per level), one
    workspace, all allocated with torch and handed to the library.  A problem
    with ``fine_boxes`` has a second level (ratio 2) whose initial state is
    given per patch (``fine_patches``) or as ``U0_fine`` over the rectangle
    starting at ``fine_lo``."""

    def __init__(self, ctx: Context, prob: W.Problem, form="batched", fixed_dt: Optional[float] = None,
                 side_stream=None):
        """side_stream: allocate and upload on this torch stream (pinned host
        memory, no host wait) and make the context's stream wait for it with
        an event, so admitting a problem does not stall work in flight."""
        torch = ctx.torch
        self.ctx, self.prob = ctx, prob
        self.form = FORMS[form] if isinstance(form, str) else int(form)
        L = lib()
        self.levels = [list(prob.boxes)] + ([list(prob.fine_boxes)] if prob.fine_boxes else [])
        arrays = []
        for boxes in self.levels:
            arr = (Box * len(boxes))()
            for b, (lo, hi) in enumerate(boxes):
                arr[b].lo[:] = list(lo)
                arr[b].hi[:] = list(hi)
            arrays.append(arr)
        self._boxes = arrays
        nl = len(self.levels)
        ptrs = (ctypes.POINTER(Box) * nl)(*[ctypes.cast(a, ctypes.POINTER(Box)) for a in arrays])
        nb = (ctypes.c_int * nl)(*[len(b) for b in self.levels])
        pid = ctypes.c_int()
        ctx.call("ctuppm_problem_create", ctypes.byref(_params(prob)), nl, ptrs, nb, ctypes.byref(pid))
        self.pid = pid.value
        dev = torch.device("cuda", torch.cuda.current_device())
        self.nv = 5 + int(prob.nspec)
        self.dev = dev
        pats = W.patch_list(prob) if nl == 2 else None
        if nl == 2:  # the fine patches, and their bounding box
            self._set_patches([(tuple(lo), tuple(U.shape[1:][::-1])) for lo, U in pats])
        if side_stream is None:
            self.lv = [self._alloc_level(boxes) for boxes in self.levels]
            self._bind_workspace()
            self.upload(prob.U0, patches=pats)
        else:
            compute = ctx.stream
            with torch.cuda.stream(side_stream):
                self.lv = [self._alloc_level(boxes) for boxes in self.levels]
                ws = self._alloc_workspace()
                self._fill_fabs(prob.U0, pats, pinned=True)
            ev = torch.cuda.Event()
            ev.record(side_stream)
            compute.wait_event(ev)
            for t in [ws] + [L[k] for L in self.lv for k in ("A", "B")]:
                t.record_stream(compute)  # freed memory is reused only after the context's work
            self.ctx.call("ctuppm_bind_workspace", self.pid, ctypes.c_void_p(ws.data_ptr()), ws.numel())
            self.ws = ws
            for level in range(len(self.lv)):
                self._bind(level)
        self.fixed_dt = float(fixed_dt) if fixed_dt else None
        self.steps_before = 0  # steps taken before a checkpoint this solver resumed from
        if fixed_dt:
            ctx.call("ctuppm_set_fixed_dt", self.pid, float(fixed_dt))

    def _alloc_level(self, boxes):
        torch = self.ctx.torch
        offsets, shapes, off = [], [], 0
        for lo, hi in boxes:
            n = [hi[d] - lo[d] + 1 for d in range(3)]
            shape = (self.nv, n[2] + 2 * NG, n[1] + 2 * NG, n[0] + 2 * NG)
            offsets.append(off)
            shapes.append(shape)
            off += (int(np.prod(shape)) + 31) // 32 * 32
        A = torch.full((off,), float("nan"), dtype=torch.float64, device=self.dev)
        B = torch.full((off,), float("nan"), dtype=torch.float64, device=self.dev)
        return {"boxes": boxes, "offsets": offsets, "shapes": shapes, "total": off, "A": A, "B": B}

    def _bind_workspace(self):
        ws = self._alloc_workspace()
        self.ctx.call("ctuppm_bind_workspace", self.pid, ctypes.c_void_p(ws.data_ptr()), ws.numel())
        self.ws = ws  # the old workspace (records copied from it on the stream) is released after the bind

    def _alloc_workspace(self):
        ws = ctypes.c_size_t()
        best = 0
        if len(self.levels) == 2:
            forms = (FORM_BATCHED,)
        elif self.form == FORM_WAVES:  # the workspace scales with the wave, not the level
            forms = (FORM_PER_BOX, FORM_WAVES)
        else:
            forms = (FORM_PER_BOX, FORM_BATCHED)
        for f in forms:
            self.ctx.call("ctuppm_workspace_bytes", self.pid, f, ctypes.byref(ws))
            best = max(best, ws.value)
        return self.ctx.torch.empty((max(best, 256),), dtype=self.ctx.torch.uint8, device=self.dev)

    def meta_bytes(self) -> int:
        """Bytes at the start of the workspace holding the library's device tables."""
        v = ctypes.c_size_t()
        self.ctx.call("ctuppm_workspace_meta_bytes", self.pid, ctypes.byref(v))
        return v.value

    # backwards-compatible views of level 0
    @property
    def UA(self):
        return self.lv[0]["A"]

    @property
    def UB(self):
        return self.lv[0]["B"]

    def _bind(self, level: int):
        L = self.lv[level]
        nb = len(L["boxes"])
        a = (ctypes.c_void_p * nb)(*[L["A"].data_ptr() + 8 * o for o in L["offsets"]])
        b = (ctypes.c_void_p * nb)(*[L["B"].data_ptr() + 8 * o for o in L["offsets"]])
        self.ctx.call("ctuppm_bind_state", self.pid, level, a, b)

    def _set_patches(self, patches):
        """Fine patches as (fine index lo, extent); the bounding box of them all."""
        self.patches = [(tuple(lo), tuple(n)) for lo, n in patches]
        lo = [min(p[0][d] for p in self.patches) for d in range(3)]
        hi = [max(p[0][d] + p[1][d] for p in self.patches) for d in range(3)]
        self.fine_lo = tuple(lo)
        self.fine_n = tuple(hi[d] - lo[d] for d in range(3))

    def upload(self, Uvalid: np.ndarray, Ufine: Optional[np.ndarray] = None, patches=None):
        """Copy a level-0 state (5 + nspec, nz, ny, nx) and the fine level's
        state (the array Ufine over the fine bounding box, or per patch a
        (fine index lo, state) pair) into the A fabs; ghosts NaN."""
        fine = patches if patches is not None else (
            [(self.fine_lo, Ufine)] if Ufine is not None and len(self.lv) == 2 else None)
        self._fill_fabs(Uvalid, fine)
        for level in range(len(self.lv)):
            self._bind(level)

    def _fill_fabs(self, Uvalid, fine, pinned: bool = False):
        """A fabs <- the state (ghosts NaN), B fabs <- NaN, on the current torch
        stream; pinned: through pinned host memory without a host wait."""
        torch = self.ctx.torch
        for level in range(len(self.lv)):
            L = self.lv[level]
            host = np.full(L["total"], np.nan)
            for box, off, shape in zip(L["boxes"], L["offsets"], L["shapes"]):
                if level == 0:
                    U, origin = Uvalid, (0, 0, 0)
                else:
                    origin, U = fine[W.patch_of_box(fine, box)]
                if U.shape[0] != self.nv:
                    raise ValueError(f"state has {U.shape[0]} components, the problem {self.nv}")
                host[off:off + int(np.prod(shape))] = W.grown_fab(U, box, origin=origin).ravel()
            t = torch.from_numpy(host)
            if pinned:
                L["A"].copy_(t.pin_memory(), non_blocking=True)
            else:
                L["A"].copy_(t)
            L["B"].fill_(float("nan"))

    def step(self, nsteps: int = 1, form=None):
        f = self.form if form is None else (FORMS[form] if isinstance(form, str) else int(form))
        self.ctx.step([self], f, nsteps)

    def step_checked(self, form=None) -> int:
        """One step with the retry criterion; the number of halvings of dt its
        deepest retry used (0: accepted at once).  Raises Rejected when even an
        eighth of the step fails (the state is then the last accepted one)."""
        f = self.form if form is None else (FORMS[form] if isinstance(form, str) else int(form))
        r = ctypes.c_int()
        self.ctx.call("ctuppm_step_checked", self.pid, f, ctypes.byref(r))
        return int(r.value)

    def step_guarded(self, nsteps: int = 1, form=None):
        """Guarded steps (no synchronisation): a failing step is not committed."""
        f = self.form if form is None else (FORMS[form] if isinstance(form, str) else int(form))
        self.ctx.step([self], f, nsteps, guarded=True)

    def rejections_seen(self) -> int:
        """Guarded steps rejected as far as the host sees without a sync."""
        v = ctypes.c_longlong()
        self.ctx.call("ctuppm_rejections_seen", self.pid, ctypes.byref(v))
        return int(v.value)

    def rejections(self) -> int:
        """Guarded steps rejected so far (synchronises; acknowledges them)."""
        v = ctypes.c_longlong()
        self.ctx.call("ctuppm_rejections", self.pid, ctypes.byref(v))
        return int(v.value)

    # a step in pieces, in the paper's order: ghost fill, dt, advance per level,
    # average down, reflux (the graph form is the whole step's, pieces run batched)
    def _piece_form(self, form) -> int:
        if form is None:
            single = len(self.levels) == 1
            form = self.form if single and self.form in (FORM_PER_BOX, FORM_WAVES) else FORM_BATCHED
        return FORMS[form] if isinstance(form, str) else int(form)

    def fill_ghosts(self, level: int = 0, form=None):
        self.ctx.call("ctuppm_fill_ghosts", self.pid, int(level), self._piece_form(form))

    def compute_dt(self, out=None, form=None):
        """dt of the next step from the CFL condition, kept for the next
        advance and written into `out` (a one-element float64 device tensor)
        when given."""
        ptr = ctypes.c_void_p(out.data_ptr()) if out is not None else None
        self.ctx.call("ctuppm_compute_dt", self.pid, self._piece_form(form), ptr)

    def advance_level(self, level: int = 0, dt=None, form=None):
        """Advance one level; dt None (the computed dt) or a one-element
        float64 device tensor (level 0 only)."""
        ptr = ctypes.c_void_p(dt.data_ptr()) if dt is not None else None
        self.ctx.call("ctuppm_advance_level", self.pid, int(level), self._piece_form(form), ptr)

    def average_down(self):
        self.ctx.call("ctuppm_average_down", self.pid)

    def reflux(self):
        self.ctx.call("ctuppm_reflux", self.pid)

    def step_in_pieces(self, nsteps: int = 1, form=None, dt=None):
        """nsteps steps, each taken piece by piece; dt None (CFL) or a device tensor."""
        for _ in range(nsteps):
            self.fill_ghosts(0, form)
            if dt is None:
                self.compute_dt(form=form)
            self.advance_level(0, dt, form)
            if len(self.levels) == 2:
                for _sub in range(2):
                    self.fill_ghosts(1, form)
                    self.advance_level(1, None, form)
                self.average_down()
                self.reflux()

    def checkpoint(self, path: str):
        """Save the current state of every level and the problem (see
        checkpoint.py), with the steps taken since the run began."""
        from . import checkpoint
        two = len(self.levels) == 2
        checkpoint.save(path, self.prob, self.state(), self.state_fine() if two else None,
                        self.fine_lo if two else None, self.levels[1] if two else None,
                        steps_taken=self.steps_before + int(self.counters()[5]), fixed_dt=self.fixed_dt)

    @classmethod
    def resume(cls, ctx: Context, path: str, form="batched") -> "Solver":
        """A solver whose state is the one saved in `path`."""
        from . import checkpoint
        prob, meta = checkpoint.load(path)
        s = cls(ctx, prob, form=form, fixed_dt=meta["fixed_dt"])
        s.steps_before = meta["steps_taken"]
        return s

    STAGE_ARRAYS = (["q", "phi"] + [f"ql{d}" for d in range(3)] + [f"qr{d}" for d in range(3)] +
                    [f"fn{d}" for d in range(3)] + [f"f1{p}" for p in range(6)] + [f"ff{d}" for d in range(3)])

    def stage_array(self, box: int, name: str, level: int = 0, form=None) -> np.ndarray:
        """An intermediate array of one box as the last step left it (names as
        in STAGE_ARRAYS), shaped (components, nz', ny', nx') over the grown box
        (q) or cells -1..n (the others)."""
        torch = self.ctx.torch
        f = self.form if form is None else (FORMS[form] if isinstance(form, str) else int(form))
        f = FORM_BATCHED if f == FORM_GRAPH else f
        a = self.STAGE_ARRAYS.index(name)
        n = ctypes.c_longlong()
        self.ctx.call("ctuppm_debug_stage", self.pid, level, box, a, f, None, ctypes.byref(n))
        out = torch.empty((n.value,), dtype=torch.float64, device=self.dev)
        self.ctx.call("ctuppm_debug_stage", self.pid, level, box, a, f, ctypes.c_void_p(out.data_ptr()),
                      ctypes.byref(n))
        lo, hi = self.levels[level][box]
        e = [hi[d] - lo[d] + 1 for d in range(3)]
        g = 2 * NG if a == 0 else 2
        shape = (-1, e[2] + g, e[1] + g, e[0] + g)
        return out.cpu().numpy().reshape(shape)

    def set_fail_hook(self, step_index: int):
        self.ctx.call("ctuppm_set_fail_hook", self.pid, int(step_index))

    def current(self) -> int:
        w = ctypes.c_int()
        self.ctx.call("ctuppm_current_state", self.pid, ctypes.byref(w))
        return w.value

    def fabs(self, level: int = 0) -> List[np.ndarray]:
        L = self.lv[level]
        # the fine level takes two substeps per step and is back in its A fabs
        which = self.current() if level == 0 else 0
        t = (L["A"] if which == 0 else L["B"]).cpu().numpy()
        return [t[o:o + int(np.prod(s))].reshape(s) for o, s in zip(L["offsets"], L["shapes"])]

    def state(self) -> np.ndarray:
        """Valid cells of the current level-0 state, (5 + nspec, nz, ny, nx)."""
        return W.gather_valid(self.fabs(0), self.prob.boxes, self.prob.n)

    def state_fine(self) -> np.ndarray:
        """Valid cells of the fine level's current state over the bounding box
        of its boxes (NaN where no fine box lies)."""
        return W.gather_valid(self.fabs(1), self.levels[1], self.fine_n, origin=self.fine_lo)

    def state_patches(self) -> List[np.ndarray]:
        """The fine level's current state, one array per patch."""
        fabs = self.fabs(1)
        out = []
        for lo, n in self.patches:
            sel = [q for q, b in enumerate(self.levels[1])
                   if all(lo[d] <= b[0][d] and b[1][d] < lo[d] + n[d] for d in range(3))]
            out.append(W.gather_valid([fabs[q] for q in sel], [self.levels[1][q] for q in sel], n, origin=lo))
        return out

    def tag(self, threshold: float) -> np.ndarray:
        """Level-0 refinement tags (nz, ny, nx) from the density-jump criterion."""
        torch = self.ctx.torch
        nx, ny, nz = self.prob.n
        t = torch.zeros((nx * ny * nz,), dtype=torch.uint8, device=self.dev)
        self.ctx.call("ctuppm_tag", self.pid, float(threshold), ctypes.c_void_p(t.data_ptr()))
        return t.cpu().numpy().reshape(nz, ny, nx).astype(bool)

    def regrid(self, fine_boxes: Sequence[W.Box], patches=None):
        """Move the fine level onto new boxes: new fabs, the new fine state
        computed on the device, the workspace re-bound.  ``patches``: the
        rectangles (fine index lo, extent) the boxes tile, for state_patches
        (default: each box its own patch)."""
        boxes = [tuple(map(tuple, b)) for b in fine_boxes]
        arr = (Box * len(boxes))()
        for b, (lo, hi) in enumerate(boxes):
            arr[b].lo[:] = list(lo)
            arr[b].hi[:] = list(hi)
        L = self._alloc_level(boxes)
        nb = len(boxes)
        a = (ctypes.c_void_p * nb)(*[L["A"].data_ptr() + 8 * o for o in L["offsets"]])
        b_ = (ctypes.c_void_p * nb)(*[L["B"].data_ptr() + 8 * o for o in L["offsets"]])
        self.ctx.call("ctuppm_regrid", self.pid, arr, nb, a, b_)
        old = self.lv[1]
        self.lv[1] = L
        self.levels[1] = boxes
        self._boxes[1] = arr
        self._set_patches(patches if patches is not None else
                          [(b[0], tuple(b[1][d] - b[0][d] + 1 for d in range(3))) for b in boxes])
        self._bind_workspace()
        del old

    def dt(self) -> float:
        v = ctypes.c_double()
        self.ctx.call("ctuppm_get_dt", self.pid, ctypes.byref(v))
        return v.value

    def counters(self) -> np.ndarray:
        c = (ctypes.c_longlong * 6)()
        self.ctx.call("ctuppm_status", self.pid, c)
        return np.array(c[:])

    def stage_bytes(self) -> Dict[str, float]:
        out = {}
        v = ctypes.c_double()
        for s, name in enumerate(stage_names()):
            self.ctx.call("ctuppm_stage_bytes", self.pid, s, ctypes.byref(v))
            out[name] = v.value
        return out

    def close(self):
        if getattr(self, "pid", None) is not None and self.ctx.h:
            self.ctx._L.ctuppm_problem_destroy(self.ctx.h, self.pid)
            self.pid = None
