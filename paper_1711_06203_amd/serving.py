"""Continuous-batching server of independent hydro problems on one GPU.

Requests (a problem and a step count) arrive over time.  The server admits
waiting requests in arrival order whenever the HBM budget has room for their
state and workspace, keeps every admitted problem resident on the device,
advances all active problems together (one batched launch set per step, each
problem with its own dt from its own CFL condition), and retires a problem as
soon as its steps are done: its state is copied back and its memory freed,
which makes room for the next arrivals.  Latency is measured on the host from
arrival to result.

Nothing here waits for the GPU in the common case.  A new problem's memory is
allocated and its initial state uploaded from pinned host memory on a side
stream, which the step stream waits for with an event; its device tables
are written by the library's asynchronous copies.  Steps are guarded (a
step whose new state fails is not committed, the retry criterion of the
paper's section 3.2); the host learns of a rejection from host-mapped memory
and only then synchronises, redoing that problem's step in halves.  A problem
is done when the event recorded after its last step has passed; the host
keeps at most two steps in flight ahead of it.

All device work goes through the C ABI (``ctuppm.Context.step`` over the
active problems); this module only schedules.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import ctuppm
from . import workloads as W

NG = 4


def footprint_bytes(prob: W.Problem) -> int:
    """Device bytes a resident problem needs: two fabs per box plus the
    batched-form stage workspace (q with 6 + nspec components on the grown box,
    phi and 18 halo-1 arrays of 5 + nspec components, plus the Runge-Kutta
    stage fabs of the method-of-lines schemes)."""
    total = 0
    nv = 5 + int(prob.nspec)
    stage_fabs = {0: 0, 1: 1, 2: 2}[ctuppm.scheme_id(prob)]  # Runge-Kutta stage fabs (MOL)
    for lo, hi in prob.boxes:
        n = [hi[d] - lo[d] + 1 for d in range(3)]
        grown = (n[0] + 2 * NG) * (n[1] + 2 * NG) * (n[2] + 2 * NG)
        h1 = ((n[0] + 2) * (n[1] + 2) + 15) // 16 * 16 * (n[2] + 2)  # halo-1 planes padded to 16 doubles
        total += 2 * nv * grown * 8 + (((nv + 1) * grown + (1 + 18 * nv) * h1) * 8 + 255) // 256 * 256
        total += stage_fabs * ((nv * grown * 8 + 255) // 256 * 256)
    return total


@dataclasses.dataclass
class Request:
    rid: int
    prob: W.Problem
    arrival: float          # seconds after the start of the run
    steps: int
    fail_step: Optional[int] = None  # test hook: the update flags a failed cell at this step, once


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: float
    finished: float
    state: Optional[np.ndarray]
    steps: int
    rejected: int = 0       # guarded steps the retry criterion rejected (redone in halves)
    failed: bool = False    # even an eighth of a step failed: the state is the last accepted one

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    def __init__(self, ctx: ctuppm.Context, hbm_budget: float = 64e9, form: str = "batched",
                 keep_states: bool = False, max_active: Optional[int] = None, inflight: int = 2,
                 async_admission: bool = True):
        """async_admission False: each admission uploads on the step stream and
        waits for it (a comparison point for the side-stream admission)."""
        self.ctx = ctx
        self.budget = float(hbm_budget)
        self.form = form
        self.keep_states = keep_states
        self.max_active = max_active
        self.inflight = inflight
        self.used = 0
        self.active: List[dict] = []
        self.finishing: List[dict] = []
        self.results: Dict[int, Result] = {}
        self.batch_sizes: List[int] = []
        self.zone_updates = 0
        self.steps_events: List = []
        self.async_admission = async_admission
        self.admit_s: List[float] = []  # host time of each admission

    def _admit(self, req: Request, now: float) -> None:
        t0 = time.perf_counter()
        if self.async_admission:
            solver = ctuppm.Solver(self.ctx, req.prob, form=self.form, side_stream=self.ctx.side_stream)
        else:
            solver = ctuppm.Solver(self.ctx, req.prob, form=self.form)
            self.ctx.torch.cuda.current_stream().synchronize()
        self.admit_s.append(time.perf_counter() - t0)
        if req.fail_step is not None:
            solver.set_fail_hook(req.fail_step)
        need = footprint_bytes(req.prob)
        self.used += need
        self.active.append({"req": req, "solver": solver, "done": 0, "need": need, "admitted": now,
                            "rejected": 0, "failed": False})

    def _retire(self, slot: dict, now_fn: Callable[[], float]) -> None:
        s = slot["solver"]
        state = s.state() if self.keep_states else None
        req = slot["req"]
        self.results[req.rid] = Result(req.rid, req.prob.n[0], req.arrival, slot["admitted"], now_fn(), state,
                                       slot["done"], slot["rejected"], slot["failed"])
        s.close()
        del slot["solver"]
        self.used -= slot["need"]

    def _resolve(self, a: dict) -> bool:
        """Synchronise and count the problem's committed steps; when a guarded
        step of it was rejected, redo the interval with the checked step
        (halving dt).  True if the problem has new rejections."""
        s = a["solver"]
        before = a["rejected"]
        a["rejected"] = s.rejections()  # synchronises, acknowledges
        a["done"] = int(s.counters()[5])
        if a["rejected"] > before and a["done"] < a["req"].steps:
            try:
                s.step_checked()
            except ctuppm.Rejected:
                a["failed"] = True
                a["done"] = a["req"].steps
                return True
            a["done"] = int(s.counters()[5])
        return a["rejected"] > before

    def _resolve_rejections(self) -> None:
        for a in self.active:
            self._resolve(a)

    def run(self, requests: Sequence[Request], realtime: bool = True) -> Dict[int, Result]:
        """Serve the requests; with realtime, arrivals follow the wall clock."""
        torch = self.ctx.torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = time.perf_counter()
        now = (lambda: time.perf_counter() - t0) if realtime else (lambda: float("inf"))
        stamp = now if realtime else (lambda: 0.0)
        qi = 0
        while qi < len(pending) or self.active or self.finishing:
            t = now()
            # admission: FIFO while the budget (and slot cap) allows
            while qi < len(pending) and pending[qi].arrival <= t:
                req = pending[qi]
                need = footprint_bytes(req.prob)
                if need > self.budget:
                    raise ValueError(f"request {req.rid} needs {need} B, above the HBM budget")
                if self.used + need > self.budget:
                    break
                if self.max_active is not None and len(self.active) >= self.max_active:
                    break
                self._admit(req, t if realtime else 0.0)
                qi += 1
            # results whose last step has run on the device (a problem whose
            # in-flight steps were rejected goes back to the active set)
            done = [f for f in self.finishing if f["event"].query()]
            self.finishing = [f for f in self.finishing if f not in done]
            for f in done:
                if f["solver"].rejections_seen() != f["rejected"]:
                    self._resolve(f)
                    if f["done"] < f["req"].steps:
                        self.active.append(f)
                        continue
                self._retire(f, stamp)
            if not self.active:
                if self.finishing:
                    self.finishing[0]["event"].synchronize()
                elif qi < len(pending) and realtime:
                    time.sleep(max(0.0, min(pending[qi].arrival - now(), 0.01)))
                continue
            # one guarded step of every active problem, batched
            solvers = [a["solver"] for a in self.active]
            try:
                self.ctx.step(solvers, self.form, 1, guarded=True)
            except ctuppm.Rejected:
                self._resolve_rejections()
            else:
                self.batch_sizes.append(len(solvers))
                for a in self.active:
                    a["done"] += 1
                    self.zone_updates += a["req"].prob.zones
            ev = torch.cuda.Event()
            ev.record(self.ctx.stream)
            self.steps_events.append(ev)
            if len(self.steps_events) > self.inflight:
                self.steps_events.pop(0).synchronize()
            for a in self.active:
                if a["done"] >= a["req"].steps:
                    a["event"] = ev
                    self.finishing.append(a)
            self.active = [a for a in self.active if a["done"] < a["req"].steps]
        torch.cuda.synchronize()
        return self.results


def poisson_requests(n_requests: int, rate: float, seed: int, steps: int = 50,
                     sizes: Sequence[int] = W.SERVING_SIZES) -> List[Request]:
    """Requests with exponential inter-arrival times (rate per second), sizes
    uniform over ``sizes`` and smooth random initial states, all seeded."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests) if rate > 0 else np.zeros(n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(n_requests):
        n = int(sizes[int(rng.integers(len(sizes)))])
        prob = W.serving_request(seed=seed * 100003 + r, n=n, steps=steps)
        out.append(Request(r, prob, float(arrivals[r]), steps))
    return out


def latency_stats(results: Dict[int, Result]) -> dict:
    lat = np.array([r.latency for r in results.values()])
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max()), "count": int(lat.size)}
