"""Benchmark: zone-updates/s of the FP64 unsplit CTU/PPM advance on one MI355X.

Workload: the 256^3 periodic Kelvin-Helmholtz shear layer split into 64 boxes
of 64^3 (gamma 5/3, CFL 0.5), stepped in the graph form (one persistent
launch per stage over all boxes, the step replayed from a hipGraph).  A step
is one pass of the whole hot path: ghost fill, CFL dt, cons->prim,
flattening, PPM + tracing, normal HLLC fluxes, both transverse stages and the
conservative update.  Inputs are resident in HBM before the timed region.

Prints one JSON line with the metric, the per-box and batched forms beside
the graph form, the roofline of the dominant kernel (algorithmic bytes per
launch over its event-timed average duration, against 8 TB/s, with what a
plain copy, reduction and fill reach in the same run beside it) and the CPU
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


def kernel_source_hash() -> str:
    """Hash of the HIP sources, to tell whether a stored counter summary was
    taken on the kernels that run now."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1711_06203_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the plain-copy calibration),
    or None when there is none for this workload or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    v = vals.get(f"bytes_per_launch[{kernel}]")
    return float(v) if v else None


def attainable_bandwidth(torch, gib: int = 2) -> dict:
    """What plain streaming kernels reach on this GPU in the same run: a device
    copy, a full reduction (read) and a fill (write) over `gib` GiB of FP64,
    10 launches each, timed with events on the current stream."""
    n = (gib << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn, moved in (("copy", lambda: b.copy_(a), 2 * n * 8), ("read", lambda: a.sum(), n * 8),
                            ("write", lambda: b.fill_(1.0), n * 8)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        e1.synchronize()
        out[name] = moved / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    out["unit"] = "GB/s"
    out["how"] = f"torch copy_ / sum / fill_ over {gib} GiB FP64, 10 launches each, HIP events"
    return out


def host_cpu() -> dict:
    """Model name and core counts of the host (lscpu, else /proc/cpuinfo)."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    model = info.get("Model name")
    if model is None and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    def num(k):
        try:
            return int(info[k])
        except (KeyError, ValueError):
            return None
    sockets, cores, tpc = num("Socket(s)"), num("Core(s) per socket"), num("Thread(s) per core")
    return {"cpu_model": model, "sockets": sockets, "physical_cores": sockets * cores if sockets and cores else None,
            "threads_per_core": tpc, "logical_cpus": num("CPU(s)"),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def measured_valu(kernel: str, workload: str):
    """VALU wave-instructions per launch of `kernel` from the committed
    rocprofv3 SQ counter summary, or None when the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    v = vals.get(f"valu_insts_per_launch[{kernel}]")
    return float(v) if v else None


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
    out = {"value": n ** 3 * reps / el, "unit": "zone-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{reps} advances of one 64^3 box (72^3 grown) of the 256^3 KH initial state "
                     f"({prob.nspec} species), "
                     f"{el:.1f} s wall, OpenMP threads={threads}"}
    out.update(host_cpu())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="kh256", choices=["kh256", "sod32", "rt384", "cloud256", "serving"],
                    help="kh256: 256^3 KH in 64 boxes of 64^3 (default); sod32: 32^3 Sod, one box; rt384: "
                         "384^3 RT in seeded uneven boxes; cloud256: two-level cloud in a Mach-2 wind; serving: "
                         "Poisson stream of independent problems")
    ap.add_argument("--nspec", type=int, default=0,
                    help="passive species advected with the flow (kh256, rt384, cloud256; the paper's GPU "
                         "proxy advects 13)")
    ap.add_argument("--scheme", default="ctu", choices=["ctu", "mol2", "mol3"],
                    help="ctu: unsplit CTU/PPM (default); mol2 / mol3: the method-of-lines formulation of the "
                         "paper's GPU proxy with SSP-RK2 / RK3 (single-level workloads)")
    ap.add_argument("--riemann", default="hllc", choices=["hllc", "twoshock"],
                    help="interface flux: HLLC (default) or the two-shock approximate Riemann solver")
    ap.add_argument("--limiter", default="cw84", choices=["cw84", "cs"],
                    help="PPM limiter: Colella & Woodward 1984 (default) or Colella & Sekora 2008")
    ap.add_argument("--regrid", type=float, default=0.0, metavar="THRESHOLD",
                    help="cloud256: after timing, tag (density jump > THRESHOLD), cluster and regrid once, and "
                         "report the time of each part")
    ap.add_argument("--steepen", action="store_true", help="CW84 contact steepening of the density")
    ap.add_argument("--concurrent-graph", action="store_true",
                    help="graph form with the three directions of each phase on three streams (default: one chain)")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--box", type=int, default=64)
    ap.add_argument("--form", default="graph", choices=["per_box", "batched", "graph", "waves"])
    ap.add_argument("--wave-boxes", type=int, default=64,
                    help="waves form: boxes per wave (the workspace holds this many boxes' stage scratch)")
    ap.add_argument("--requests", type=int, default=200, help="serving: requests per arrival rate")
    ap.add_argument("--no-serving", action="store_true",
                    help="kh256: skip the serving leg (a Poisson stream at 0.8 of the batched capacity, served "
                         "batched and per box)")
    ap.add_argument("--serving-requests", type=int, default=500, help="requests of the serving leg")
    ap.add_argument("--tune", action="store_true", help="autotune launch shapes before timing")
    ap.add_argument("--tune-stages", action="store_true",
                    help="autotune the planes per work unit of each stage before timing")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--skip-forms", action="store_true", help="time only the requested form")
    ap.add_argument("--print-hash", action="store_true", help="print the kernel source hash and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 10 plain device copies of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.print_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the box decomposition would shard across GPUs, one halo exchange and one dt reduction per step)",
              file=sys.stderr)
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
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "sod32":
        prob = W.sod(n=32, steps=20)
        args.form = "per_box" if args.form == "graph" and "--form" not in sys.argv else args.form
        wname = "sod_32^3_single_box_outflow_x"
    elif args.workload == "rt384":
        prob = W.rayleigh_taylor(n=384, nspec=args.nspec)
        wname = f"rayleigh_taylor_384^3_{len(prob.boxes)}_uneven_boxes_gz-1"
    elif args.workload == "cloud256":
        prob = W.cloud_wind(n=256, box=64, fine_box=32, nspec=args.nspec)
        args.form = "batched" if args.form == "per_box" else args.form
        wname = "cloud_wind_two_level_256^3_64x64^3_fine_256^3_512x32^3"
    else:
        prob = W.kelvin_helmholtz(n=args.n, box=args.box, nspec=args.nspec)
        wname = f"kelvin_helmholtz_{args.n}^3_{(args.n // args.box) ** 3}x{args.box}^3_periodic"
    if args.nspec and args.workload != "sod32":
        wname += f"_{args.nspec}_species"
    if args.scheme != "ctu":
        if prob.fine_boxes is not None:
            print("the method-of-lines schemes are single-level", file=sys.stderr)
            sys.exit(2)
        prob.scheme = ctuppm.SCHEMES[args.scheme]
        wname += f"_{args.scheme}"
    if args.riemann != "hllc":
        prob.riemann = ctuppm.RIEMANN[args.riemann]
        wname += f"_{args.riemann}"
    if args.limiter != "cw84":
        prob.limiter = ctuppm.LIMITERS[args.limiter]
        wname += f"_{args.limiter}"
    if args.steepen:
        prob.steepen = 1
        wname += "_steepened"
    # key of the stored counter summary of this workload
    tkey = args.workload + (f"s{args.nspec}" if args.nspec else "") + ("" if args.scheme == "ctu" else args.scheme) + (
        "" if args.riemann == "hllc" else args.riemann) + ("" if args.limiter == "cw84" else args.limiter) + (
        "steep" if args.steepen else "")
    ctx = ctuppm.Context()
    if args.concurrent_graph:
        ctx.set_concurrency(True)
    waves = args.form == "waves"
    if waves:
        if prob.fine_boxes is not None:
            print("the waves form is single-level", file=sys.stderr)
            sys.exit(2)
        ctx.set_wave_boxes(args.wave_boxes)
    solver = ctuppm.Solver(ctx, prob, form=args.form)
    two_level = prob.fine_boxes is not None
    # zone-updates per step: the fine level takes two substeps per coarse step
    zones = prob.zones + (2 * sum(int(U[0].size) for _, U in W.patch_list(prob)) if two_level else 0)
    tuning = None
    if args.tune:
        from paper_1711_06203_amd import autotune
        tuning = autotune.tune(ctx, [solver], steps=3, cache=None)
        solver.upload(prob.U0, patches=W.patch_list(prob) if two_level else None)
    stage_tuning = None
    if args.tune_stages:
        from paper_1711_06203_amd import autotune
        stage_tuning = autotune.tune_stages(ctx, [solver], steps=3, cache=None)
        solver.upload(prob.U0, patches=W.patch_list(prob) if two_level else None)

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
        if (two_level and f == "per_box") or waves:  # a waves-sized workspace holds no batched scratch
            continue
        if f not in forms and not args.skip_forms:
            k = max(3, args.steps // 5)
            forms[f] = zones * k / timed(f, k, 1)

    # dominant kernel: event-timed stage launches of the batched form (the same
    # kernels and grids the graph replays), on the stream they run on
    tsteps = max(3, args.steps // 5)
    ctx.set_timing(True)
    solver.step(tsteps, form="waves" if waves else "batched")
    ctx.set_timing(False)
    st = ctx.stage_times()
    sbytes = solver.stage_bytes()
    stage_avg = {k: (ms / n if n else 0.0) for k, (ms, n) in st.items()}
    dom = max(st, key=lambda k: st[k][0])
    avg_ms = stage_avg[dom]
    launches_per_step = st[dom][1] / tsteps
    # algorithmic bytes of the stage per step over its launch time per step
    achieved = sbytes[dom] / (avg_ms * launches_per_step * 1e-3) / 1e9
    traffic = measured_traffic(dom, tkey)
    # the whole step: measured HBM bytes of every stage (per launch, times its
    # launches per step) over the timed step
    step_bytes = 0.0
    for k, (ms, n) in st.items():
        if n:
            b = measured_traffic(k, tkey)
            if b is None:
                step_bytes = None
                break
            step_bytes += b * n / tsteps
    step_roof = None
    if step_bytes:
        step_gbs = step_bytes / (el / args.steps) / 1e9
        step_roof = {"measured_bytes": step_bytes, "achieved": step_gbs, "frac": step_gbs / HBM_PEAK_GBS,
                     "how": "sum over stages of rocprofv3 bytes per launch x launches per step, over ms_per_step"}
    cnt = solver.counters()
    regrid_info = None
    if args.regrid > 0.0 and two_level:
        from paper_1711_06203_amd import regrid
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tags = solver.tag(args.regrid)
        t1 = time.perf_counter()
        patches = regrid.patches_from_tags(tags, buffer=2)
        t2 = time.perf_counter()
        boxes, rects = regrid.fine_level(patches, 32) if patches else (None, None)
        if boxes:
            solver.regrid(boxes, rects)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        solver.step(1)
        torch.cuda.synchronize()
        regrid_info = {"threshold": args.regrid, "tagged_cells": int(tags.sum()), "patches": patches,
                       "fine_boxes": len(boxes) if boxes else 0, "tag_ms": (t1 - t0) * 1e3,
                       "cluster_ms": (t2 - t1) * 1e3, "regrid_ms": (t3 - t2) * 1e3,
                       "counters_after_step": [int(c) for c in solver.counters()]}
    out = {
        "metric": "zone-updates/s FP64 (unsplit CTU/PPM advance)" if args.scheme == "ctu" else
                  "zone-updates/s FP64 (method-of-lines PPM advance)",
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
        "config": {"workload": wname, "form": args.form, "zone_updates_per_step": zones, "boxes": len(prob.boxes),
                   "species": prob.nspec, "scheme": args.scheme, "riemann": args.riemann, "limiter": args.limiter, "steepen": bool(args.steepen),
                   "gamma": prob.gamma, "cfl": prob.cfl, "concurrent_graph": bool(args.concurrent_graph),
                   "wave_boxes": args.wave_boxes if waves else None, "workspace_bytes": int(solver.ws.numel()), "tuning": tuning and {k: tuning[k] for k in
                                                                               ("blocks_per_cu", "zseg", "ytile")},
                   "stage_planes": stage_tuning and stage_tuning["planes"]},
        "forms": {k: v for k, v in forms.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": sbytes[dom] / launches_per_step, "avg_launch_ms": avg_ms,
                     "whole_step": step_roof},
        "stage_ms": {k: round(v, 4) for k, v in stage_avg.items() if v},
        "counters": [int(c) for c in cnt],
    }
    if regrid_info:
        out["regrid"] = regrid_info
    # the headline rate against the method's algorithmic floor: 80 bytes per
    # zone-update (read and write the 5 conserved doubles once), or 131 with
    # the ghost cells of 64^3 boxes stored and filled
    out["roofline"]["alg_frac_80B"] = value * 80.0 / (HBM_PEAK_GBS * 1e9)
    out["roofline"]["alg_frac_131B"] = value * 131.0 / (HBM_PEAK_GBS * 1e9)
    valu = measured_valu(dom, tkey)
    out["roofline"]["valu_busy"] = (
        None if valu is None else {"frac": valu * 4.0 / (1024 * 2.4e9 * avg_ms * 1e-3), "valu_insts_per_launch": valu,
                                    "how": "rocprofv3 SQ_INSTS_VALU per launch x 4 cycles / (1024 SIMDs x 2.4 GHz x "
                                           "launch time)"})
    solver.close()
    del solver
    torch.cuda.empty_cache()
    att = attainable_bandwidth(torch)
    att["probe"] = {k: ctx.bandwidth_probe(k) for k in ("copy", "read", "write")}
    att["probe"]["how"] = ("the library's streaming kernel, 16-byte accesses, grid-stride, best of 4 grids, "
                           "2 GiB FP64, 10 launches each")
    out["roofline"]["attainable"] = att
    out["roofline"]["frac_of_copy"] = achieved / max(att["copy"], att["probe"]["copy"])
    if step_roof:
        step_roof["frac_of_copy"] = step_roof["achieved"] / max(att["copy"], att["probe"]["copy"])
    if (not args.no_serving and args.workload == "kh256" and args.n == 256 and args.box == 64
            and args.scheme == "ctu" and args.riemann == "hllc" and args.limiter == "cw84" and not args.steepen):
        out["serving"] = serving_leg(ctx, args.serving_requests)
    ctx.close()
    if (not args.no_cpu and args.workload == "kh256" and args.n == 256 and args.box == 64
            and args.scheme == "ctu" and args.riemann == "hllc" and args.limiter == "cw84"
            and not args.steepen):
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def serving_leg(ctx, nreq: int) -> dict:
    """The serving workload beside the headline.  Capacity: 120 requests
    present at t = 0, served batched and, the same requests, per box (every
    stage launched per box of every problem).  Latency: one Poisson stream of
    `nreq` requests at 0.8 of the batched capacity, served batched, per box,
    and batched with synchronous admissions."""
    import numpy as np
    from paper_1711_06203_amd import serving
    out = {"workload": "serving_periodic_N^3_N_in_32-128_50_steps", "hbm_budget_bytes": 64e9,
           "capacity": {}, "load": 0.8, "requests": nreq}
    sat = serving.poisson_requests(120, rate=0.0, seed=11)
    for form in ("batched", "per_box"):
        srv = serving.Server(ctx, hbm_budget=64e9, form=form)
        t0 = time.perf_counter()
        res = srv.run(sat, realtime=True)
        el = time.perf_counter() - t0
        out["capacity"][form] = {"requests_per_s": len(res) / el, "zone_updates_per_s": srv.zone_updates / el,
                                 "mean_batch": float(np.mean(srv.batch_sizes))}
    rate = 0.8 * out["capacity"]["batched"]["requests_per_s"]
    out["arrival_rate_per_s"] = rate
    stream = serving.poisson_requests(nreq, rate=rate, seed=92)
    # the stream served batched, per box, and batched with each admission
    # uploading on the step stream and waiting for it
    for name, form, asyn in (("batched", "batched", True), ("per_box", "per_box", True),
                             ("batched_sync_admission", "batched", False)):
        srv = serving.Server(ctx, hbm_budget=64e9, form=form, async_admission=asyn)
        t0 = time.perf_counter()
        res = srv.run(stream, realtime=True)
        el = time.perf_counter() - t0
        st = serving.latency_stats(res)
        out[name] = {"zone_updates_per_s": srv.zone_updates / el, "requests_per_s": len(res) / el,
                     "p50_s": st["p50_s"], "p99_s": st["p99_s"], "mean_batch": float(np.mean(srv.batch_sizes)),
                     "admission_ms_p50": 1e3 * float(np.percentile(srv.admit_s, 50)),
                     "admission_ms_max": 1e3 * float(np.max(srv.admit_s)),
                     "rejected_steps": int(sum(r.rejected for r in res.values())), "wall_s": el}
        print(json.dumps({"serving_leg": name, **out[name]}), file=sys.stderr, flush=True)
    out["served_over_per_box"] = (out["capacity"]["batched"]["zone_updates_per_s"]
                                  / out["capacity"]["per_box"]["zone_updates_per_s"])
    return out


def bench_serving(args):
    """Poisson streams of independent periodic problems (N in {32,...,128}, 50
    steps each) at 0.5, 0.8 and 0.95 of the measured saturated capacity."""
    import numpy as np
    import torch
    from paper_1711_06203_amd import ctuppm, serving
    ctx = ctuppm.Context()
    # capacity: all requests present at t = 0 (saturated continuous batching)
    reqs = serving.poisson_requests(args.requests, rate=0.0, seed=11)
    srv = serving.Server(ctx, hbm_budget=64e9)
    t0 = time.perf_counter()
    res = srv.run(reqs, realtime=True)
    el = time.perf_counter() - t0
    capacity = len(res) / el
    lines = {"saturated": {"requests_per_s": capacity, "zone_updates_per_s": srv.zone_updates / el,
                           "mean_batch": float(np.mean(srv.batch_sizes)), **serving.latency_stats(res)}}
    for frac in (0.5, 0.8, 0.95):
        reqs = serving.poisson_requests(args.requests, rate=frac * capacity, seed=12 + int(100 * frac))
        srv = serving.Server(ctx, hbm_budget=64e9)
        t0 = time.perf_counter()
        res = srv.run(reqs, realtime=True)
        el = time.perf_counter() - t0
        lines[f"rate_{frac}"] = {"arrival_rate_per_s": frac * capacity, "zone_updates_per_s": srv.zone_updates / el,
                                 "mean_batch": float(np.mean(srv.batch_sizes)), **serving.latency_stats(res)}
        print(json.dumps({"serving": lines[f"rate_{frac}"], "frac": frac}), file=sys.stderr, flush=True)
    out = {"metric": "p50/p99 solve latency of a served stream (FP64 CTU/PPM)", "value": lines["rate_0.8"]["p99_s"],
           "unit": "s", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {"workload": "serving_periodic_N^3_N_in_32-128_50_steps",
                                            "requests_per_rate": args.requests, "hbm_budget_bytes": 64e9},
           "serving": lines}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
