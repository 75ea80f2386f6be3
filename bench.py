"""Benchmark: zone-updates/s of the FP64 unsplit CTU/PPM advance on one MI355X.

Workload: the 256^3 periodic Kelvin-Helmholtz shear layer split into 64 boxes
of 64^3 (gamma 5/3, CFL 0.5), stepped in the graph form (one persistent
launch per stage over all boxes, the step replayed from a hipGraph).  A step
is one pass of the whole hot path: ghost fill, CFL dt, cons->prim,
flattening, PPM + tracing, normal HLLC fluxes, both transverse stages and the
conservative update.  Inputs are resident in HBM before the timed region.

Prints one JSON line with the metric, the per-box and batched forms beside
the graph form, the roofline of the dominant kernel (algorithmic bytes per
launch over its event-timed average duration, against 8 TB/s) and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def cpu_baseline(prob, seconds: float = 12.0):
    """Oracle on one 64^3 box of the same initial state (ghosts from the
    filled whole-domain state), advanced repeatedly until ~`seconds` pass."""
    import numpy as np
    import oracle
    P = oracle.params_of(prob)
    G = oracle.fill_domain(oracle.grow(prob.U0), P)
    dt = P.cfl / oracle.signal_speed(G, P)
    lo = prob.boxes[0][0]
    n = 64
    box = np.ascontiguousarray(G[:, lo[2]:lo[2] + n + 8, lo[1]:lo[1] + n + 8, lo[0]:lo[0] + n + 8])
    oracle.advance_box(box, P, dt)  # warm-up (page-in, thread start)
    reps, t0 = 0, time.perf_counter()
    while True:
        oracle.advance_box(box, P, dt)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": n ** 3 * reps / el, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} advances of one 64^3 box (72^3 grown) of the 256^3 KH initial state, "
                      f"{el:.1f} s wall, OpenMP threads={threads}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--box", type=int, default=64)
    ap.add_argument("--form", default="graph", choices=["per_box", "batched", "graph"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--skip-forms", action="store_true", help="time only the requested form")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 10 plain device copies of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the box decomposition would shard across GPUs; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1711_06203_amd import ctuppm, workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8}))
        return
    prob = W.kelvin_helmholtz(n=args.n, box=args.box)
    ctx = ctuppm.Context()
    solver = ctuppm.Solver(ctx, prob, form=args.form)
    zones = prob.zones

    def timed(form, steps, warm):
        solver.step(warm, form=form)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.step(steps, form=form)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # headline: the requested form
    el = timed(args.form, args.steps, args.warmup)
    value = zones * args.steps / el
    forms = {args.form: value}
    for f in ("per_box", "batched", "graph"):
        if f not in forms and not args.skip_forms:
            k = max(3, args.steps // 5)
            forms[f] = zones * k / timed(f, k, 1)

    # dominant kernel: event-timed stage launches of the batched form
    ctx.set_timing(True)
    solver.step(max(3, args.steps // 5), form="batched")
    ctx.set_timing(False)
    st = ctx.stage_times()
    sbytes = solver.stage_bytes()
    stage_avg = {k: (ms / n if n else 0.0) for k, (ms, n) in st.items()}
    dom = max(st, key=lambda k: st[k][0])
    avg_ms = stage_avg[dom]
    achieved = sbytes[dom] / (avg_ms * 1e-3) / 1e9
    cnt = solver.counters()
    out = {
        "metric": "zone-updates/s FP64 (unsplit CTU/PPM advance)",
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"kelvin_helmholtz_{args.n}^3_{(args.n // args.box) ** 3}x{args.box}^3_periodic",
                   "form": args.form, "zones": zones, "gamma": prob.gamma, "cfl": prob.cfl},
        "forms": {k: v for k, v in forms.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": sbytes[dom], "avg_launch_ms": avg_ms},
        "stage_ms": {k: round(v, 4) for k, v in stage_avg.items() if v},
        "counters": [int(c) for c in cnt],
    }
    solver.close()
    ctx.close()
    del solver
    torch.cuda.empty_cache()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
