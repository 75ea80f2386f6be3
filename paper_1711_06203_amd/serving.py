"""Continuous-batching server of independent hydro problems on one GPU.

Requests (a problem and a step count) arrive over time.  The server admits
waiting requests in arrival order whenever the HBM budget has room for their
state and workspace, keeps every admitted problem resident on the device,
advances all active problems together (one batched launch set per step, each
problem with its own dt from its own CFL condition), and retires a problem as
soon as its steps are done: its state is copied back and its memory freed,
which makes room for the next arrivals.  Latency is measured on the host from
arrival to result.

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
        h1 = (n[0] + 2) * (n[1] + 2) * (n[2] + 2)
        total += 2 * nv * grown * 8 + (((nv + 1) * grown + (1 + 18 * nv) * h1) * 8 + 255) // 256 * 256
        total += stage_fabs * ((nv * grown * 8 + 255) // 256 * 256)
    return total


@dataclasses.dataclass
class Request:
    rid: int
    prob: W.Problem
    arrival: float          # seconds after the start of the run
    steps: int


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: float
    finished: float
    state: Optional[np.ndarray]
    steps: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    def __init__(self, ctx: ctuppm.Context, hbm_budget: float = 64e9, form: str = "batched",
                 keep_states: bool = False, max_active: Optional[int] = None):
        self.ctx = ctx
        self.budget = float(hbm_budget)
        self.form = form
        self.keep_states = keep_states
        self.max_active = max_active
        self.used = 0
        self.active: List[dict] = []
        self.results: Dict[int, Result] = {}
        self.batch_sizes: List[int] = []
        self.zone_updates = 0

    def _admit(self, req: Request, now: float) -> None:
        solver = ctuppm.Solver(self.ctx, req.prob, form=self.form)
        need = footprint_bytes(req.prob)
        self.used += need
        self.active.append({"req": req, "solver": solver, "done": 0, "need": need, "admitted": now})

    def _retire(self, slot: dict, now_fn: Callable[[], float]) -> None:
        s = slot["solver"]
        state = s.state() if self.keep_states else None
        if not self.keep_states:
            self.ctx.torch.cuda.current_stream().synchronize()
        req = slot["req"]
        self.results[req.rid] = Result(req.rid, req.prob.n[0], req.arrival, slot["admitted"], now_fn(), state,
                                       slot["done"])
        s.close()
        del slot["solver"]
        self.used -= slot["need"]

    def run(self, requests: Sequence[Request], realtime: bool = True) -> Dict[int, Result]:
        """Serve the requests; with realtime, arrivals follow the wall clock."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        t0 = time.perf_counter()
        now = (lambda: time.perf_counter() - t0) if realtime else (lambda: float("inf"))
        qi = 0
        while qi < len(pending) or self.active:
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
            if not self.active:
                if qi < len(pending) and realtime:
                    time.sleep(max(0.0, min(pending[qi].arrival - now(), 0.01)))
                continue
            # one step of every active problem, batched
            solvers = [a["solver"] for a in self.active]
            self.ctx.step(solvers, self.form, 1)
            self.batch_sizes.append(len(solvers))
            for a in self.active:
                a["done"] += 1
                self.zone_updates += a["req"].prob.zones
            finished = [a for a in self.active if a["done"] >= a["req"].steps]
            if finished:
                for a in finished:
                    self._retire(a, now if realtime else (lambda: 0.0))
                self.active = [a for a in self.active if a["done"] < a["req"].steps]
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
