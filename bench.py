"""Benchmark: phase-space cell-updates/s per sweep of the SL-MPP Strang step.

Default workload: three-dimensional electrostatic Landau damping at
48^3 x 48^3 (1.22e10 cells, 48.9 GB of FP32 f), SL-MPP7, CFL 0.2, in-place
pencil sweeps; one step = 9 sweeps (v1 v2 v3 half, x3 x2 x1, v1 v2 v3 half)
plus the FP64 velocity moment and Poisson solve.  Inputs are synthetic
(the analytic initial condition on the grid), resident in HBM before the
timed region.

Output: one JSON line on stdout.  `value` = sweeps * cells * steps / time
(whole-job throughput).  `roofline` is for the sweep kernel (the dominant
kernel), timed per launch with HIP events on the library's stream;
`cpu_baseline` is the FP64 CPU oracle on a bounded sample of the same
workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "phase-space cell-updates/s per sweep, FP32 vs FP64, % HBM peak at stated L1"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name, dtype):
    from paper_1702_08521_amd import workloads as W

    if name == "landau_3d3v":
        return W.landau_3d3v(n=48, order=7)
    if name == "jeans_3d3v":
        return W.jeans_3d3v(n=32, order=5)
    if name == "landau_nl_1d1v":
        return W.landau_nl_1d1v()
    if name == "landau_1d1v":
        return W.landau_1d1v()
    if name == "collapse_3d3v":
        return W.collapse_3d3v(nx=64, nv=32, order=5)
    if name == "ensemble":
        return None
    raise SystemExit(f"unknown workload {name}")


def read_traffic(kernel_key):
    """HBM traffic per launch from the committed counter summary, or None
    when the summary is absent or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    ent = t.get(kernel_key)
    if not ent:
        return None
    import hashlib

    src = os.path.join(ROOT, "paper_1702_08521_amd", "csrc", "sweep.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if ent.get("sweep_src_sha") != h:
        return None
    return ent.get("bytes_per_launch")


def alloc_f(S, torch, shape, tdt, dev):
    """f in physically contiguous device memory (slmpp_alloc_device: the
    strided sweeps take fewer address translations), or a torch allocation
    where the driver cannot provide such memory.  Returns (buffer or None,
    tensor, placement)."""
    import numpy as np

    nbytes = int(np.prod(shape)) * torch.empty((), dtype=tdt).element_size()
    try:
        buf = S.DeviceBuffer(nbytes, contiguous=True)
    except S.SlmppError:
        return None, torch.empty(shape, dtype=tdt, device=dev), "default"
    return buf, buf.tensor(shape, tdt, dev), "contiguous"


def release_f(torch, buf):
    torch.cuda.synchronize()
    if buf is not None:
        buf.free()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec_fn, n_nproc, n_one, repeats=5):
    """The FP64 oracle built -O3 -march=native, timed per sweep on this
    host: every axis of the workload at n_nproc^D x n_nproc^D with the
    host's thread share, and at n_one^D x n_one^D with one thread; one
    warm-up and `repeats` timed sweeps per axis, the median kept.  The cost
    per cell is flat in the grid size (pencil by pencil), so the rates stand
    for the full-size workload."""
    import statistics

    import oracle as O

    O.use_native()
    nproc = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    legs = {}
    t_all = time.perf_counter()
    for threads, n in ((nproc, n_nproc), (1, n_one)):
        O.set_threads(threads)
        s = spec_fn(n)
        grid = O.make_grid(s)
        f = O.init_separable(grid, *__import__("paper_1702_08521_amd.workloads",
                                               fromlist=["x"]).separable_factors(s))
        acc = O.field(grid, f)
        D = s["D"]
        cells = 1
        for l in range(D):
            cells *= s["nx"][l] * s["nv"][l]
        nxs = grid.n_space
        per_axis = {}
        for axis in range(2 * D):
            if axis < D:
                sweep = lambda: O.advect_x(grid, f, axis, s["dt"])  # noqa: E731
            else:
                comp = acc[(axis - D) * nxs:(axis - D + 1) * nxs]
                sweep = lambda: O.advect_v(grid, f, axis - D, 0.5 * s["dt"], comp)  # noqa: E731
            sweep()
            ts = []
            for _ in range(repeats):
                t0 = time.perf_counter()
                sweep()
                ts.append(time.perf_counter() - t0)
            name = ("x%d" % (axis + 1)) if axis < D else ("v%d" % (axis - D + 1))
            per_axis[name] = cells / statistics.median(ts)
        # a Strang step sweeps every x axis once and every v axis twice
        weights = {k: (1 if k[0] == "x" else 2) for k in per_axis}
        t_step = sum(w / per_axis[k] for k, w in weights.items())
        legs[threads] = {"grid": " x ".join(str(v) for v in list(s["nx"][:D]) + list(s["nv"][:D])),
                         "cells": cells,
                         "cell_updates_per_s": sum(weights.values()) / t_step,
                         "per_axis": {k: round(v, 1) for k, v in per_axis.items()}}
        log(f"[bench] cpu baseline {threads} thread(s) at {legs[threads]['grid']}: "
            f"{legs[threads]['cell_updates_per_s']:.3e} cell-updates/s per sweep")
    wall = time.perf_counter() - t_all
    return {
        "value": legs[nproc]["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "cores": nproc,
        "kind": "oracle",
        "sample": (f"FP64 oracle, gcc -O3 -march=native -ffp-contract=off, OpenMP over pencils, on "
                   f"{cpu_model()} ({os.cpu_count()} CPUs, {nproc} threads used); median of "
                   f"{repeats} timed sweeps after one warm-up, every axis, weighted as in a "
                   f"Strang step (x once, v twice): {nproc} threads at {legs[nproc]['grid']}, 1 thread "
                   f"at {legs[1]['grid']} (per cell, the cost being linear in cells); {wall:.1f} s"),
        "single_thread": {"value": legs[1]["cell_updates_per_s"], "cores": 1,
                          "grid": legs[1]["grid"], "per_axis": legs[1]["per_axis"]},
        "per_axis": legs[nproc]["per_axis"],
    }


def ensemble_leg(steps, warmup, dtype="f32", compare_fp64=True, log_prefix="[ensemble]"):
    """The batched ensemble: 256 independent runs of uneven sizes advanced
    together by the captured step graph, tile widths autotuned."""
    import numpy as np
    import torch

    from paper_1702_08521_amd import slmpp, workloads as W

    specs = W.ensemble()
    storage = slmpp.F32 if dtype == "f32" else slmpp.F64
    stream = torch.cuda.Stream()

    bufs = []

    def make(st, merged=False):
        # every run's f in one physically contiguous buffer (256-byte
        # aligned views), or torch allocations where the driver cannot
        # provide one
        tdt = torch.float32 if st == slmpp.F32 else torch.float64
        shapes = [tuple(s["nx"][:s["D"]]) + tuple(s["nv"][:s["D"]]) for s in specs]
        sizes = [int(np.prod(sh)) for sh in shapes]
        es = 4 if st == slmpp.F32 else 8
        q = 256 // es
        offs, total = [], 0
        for n in sizes:
            offs.append(total)
            total += (n + q - 1) // q * q
        buf, big, placement = alloc_f(slmpp, torch, (total,), tdt,
                                      torch.device("cuda", torch.cuda.current_device()))
        bufs.append((buf, placement))
        fs = [big[o:o + n].view(sh) for o, n, sh in zip(offs, sizes, shapes)]
        b = slmpp.Batch([slmpp.make_desc(dict(s, merge_kicks=merged), st) for s in specs],
                        [s["dt"] for s in specs], fs=fs, stream=stream)
        for r, s in enumerate(specs):
            sx, gv = W.separable_factors(s)
            b.init_separable(r, sx, gv)
        return b

    cells = [int(np.prod(s["nx"][:s["D"]])) * int(np.prod(s["nv"][:s["D"]])) for s in specs]
    updates = sum(c * 3 * s["D"] for c, s in zip(cells, specs))  # cell-updates per step
    b = make(storage)
    t0 = time.perf_counter()
    b.autotune(None)
    tune_s = time.perf_counter() - t0
    # algorithmic HBM bytes of a step as the library runs it: read + write
    # of f per pass (a two-axis kick pass covers two sweeps), one read for
    # the moment
    step_bytes = b.step_bytes()
    widths = {}
    for r, s in enumerate(specs):
        for a in range(2 * s["D"]):
            w = b.tile_width(r, a)
            widths[w] = widths.get(w, 0) + 1
    if warmup:
        b.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    b.step(steps)
    ev1.record(stream)
    ev1.synchronize()
    graph_ms = ev0.elapsed_time(ev1) / steps
    ev0.record(stream)
    b.step_eager(steps)
    ev1.record(stream)
    ev1.synchronize()
    eager_ms = ev0.elapsed_time(ev1) / steps
    # the same steps with every sweep in the grouped tile launch (no
    # persistent launches over runs of one geometry), for comparison
    b.set_fast_min_cells(-1)
    b.step(1)
    ev0.record(stream)
    b.step(steps)
    ev1.record(stream)
    ev1.synchronize()
    tiles_only_ms = ev0.elapsed_time(ev1) / steps
    log(f"{log_prefix} {len(specs)} runs, {sum(cells):.3e} cells, graph {graph_ms:.3f} ms/step, "
        f"eager {eager_ms:.3f} ms/step, tile launch only {tiles_only_ms:.3f} ms/step, "
        f"autotune {tune_s:.2f} s")
    out = {
        "runs": len(specs),
        "cells": sum(cells),
        "cell_updates_per_step": updates,
        "steps": steps,
        "graph_ms_per_step": round(graph_ms, 4),
        "eager_ms_per_step": round(eager_ms, 4),
        "tile_launch_only_ms_per_step": round(tiles_only_ms, 4),
        "cell_updates_per_s": updates / (graph_ms * 1e-3),
        "step_GB_s": round(step_bytes / (graph_ms * 1e-3) / 1e9, 1),
        "step_bytes": step_bytes,
        "autotune_s": round(tune_s, 3),
        "tile_widths": {str(k): v for k, v in sorted(widths.items())},
    }
    # merged kicks (SLMPP_FLAG_MERGE_KICKS on every run): 10 steps per call
    bm = make(storage, merged=True)
    bm.step(10)
    torch.cuda.synchronize()
    ncall = max(1, steps // 10)
    ev0.record(stream)
    for _ in range(ncall):
        bm.step(10)
    ev1.record(stream)
    ev1.synchronize()
    merged_ms = ev0.elapsed_time(ev1) / (10 * ncall)
    out["merged_kicks"] = {"steps_per_call": 10, "graph_ms_per_step": round(merged_ms, 4),
                           "step_body_bytes": bm.step_bytes(),
                           "step_speedup": round(graph_ms / merged_ms, 3)}
    log(f"{log_prefix} merged kicks: {merged_ms:.3f} ms/step (10 steps per call)")
    bm.close()
    if compare_fp64 and storage == slmpp.F32:
        # the same ensemble in FP64 storage from the same start, for the error
        # of FP32 storage and the FP64 rate on the same GPU
        n_cmp = 100
        b32 = make(slmpp.F32)
        b64 = make(slmpp.F64)
        b32.step(n_cmp)
        b64.autotune(None)
        b64.step(n_cmp)
        torch.cuda.synchronize()
        ev0.record(stream)
        b64.step(n_cmp)
        ev1.record(stream)
        ev1.synchronize()
        ms64 = ev0.elapsed_time(ev1) / n_cmp
        b32.step(n_cmp)
        torch.cuda.synchronize()
        worst = 0.0
        for r in range(len(specs)):
            a32, a64 = b32.get_f(r), b64.get_f(r)
            worst = max(worst, float(np.abs(a32 - a64).sum() / np.abs(a64).sum()))
        out["fp64_same_ensemble"] = {"graph_ms_per_step": round(ms64, 4),
                                     "cell_updates_per_s": updates / (ms64 * 1e-3)}
        out["fp32_vs_fp64_L1_rel_max_over_runs"] = worst
        out["fp32_vs_fp64_steps"] = 2 * n_cmp
        b32.close()
        b64.close()
    b.close()
    out["f_placement"] = bufs[0][1]
    for buf, _ in bufs:
        release_f(torch, buf)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="landau_3d3v")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=24,
                    help="grid side of the oracle's timing with the host's thread share")
    ap.add_argument("--cpu-sample-1t", type=int, default=16,
                    help="grid side of the oracle's single-thread timing")
    ap.add_argument("--cpu-steps", type=int, default=3,
                    help="oracle steps of the whole ensemble in its cpu_baseline (--workload ensemble)")
    ap.add_argument("--merge-compare", type=int, default=6,
                    help="steps in one call with merged velocity half-steps (0: skip)")
    ap.add_argument("--rk-compare", type=int, default=2,
                    help="steps of RK-MPP5 and SL-MPP5 on the same workload (0: skip)")
    ap.add_argument("--ensemble-steps", type=int, default=100,
                    help="steps of the batched ensemble reported in detail.ensemble (0: skip)")
    ap.add_argument("--fp64-compare", type=int, default=1,
                    help="1: run the same workload in FP64 storage for its rate and the FP32 error (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        raise SystemExit(2)

    import numpy as np
    import torch

    from paper_1702_08521_amd import slmpp, workloads as W

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.workload == "ensemble":
        return ensemble_main(args)
    spec = workload(args.workload, args.dtype)
    storage = slmpp.F32 if args.dtype == "f32" else slmpp.F64
    D = spec["D"]
    cells = int(np.prod(spec["nx"][:D])) * int(np.prod(spec["nv"][:D]))
    sweeps = 3 * D
    dt = spec["dt"]
    log(f"[bench] {spec['name']} cells={cells:.3e} dtype={args.dtype} steps={args.steps} warmup={args.warmup}")

    stream = torch.cuda.Stream(device=dev)
    fshape = tuple(spec["nx"][:D]) + tuple(spec["nv"][:D])
    tdt = torch.float32 if storage == slmpp.F32 else torch.float64
    f_buf, f_t, placement = alloc_f(slmpp, torch, fshape, tdt, dev)
    ctx = slmpp.Context(slmpp.make_desc(spec, storage), f=f_t, stream=stream, device=dev)
    s, gv = W.separable_factors(spec)
    ctx.init_f_separable(s, gv)
    ctx.field()
    ctx.sync()
    diag0 = ctx.diag()
    log("[bench] initialised")
    if args.warmup > 0:
        ctx.step(dt, args.warmup)
    ctx.sync()
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(dt, args.steps)
    ctx.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tim = ctx.timing_read()
    ctx.timing_enable(False)
    no_events_ms = None
    if cells < (1 << 24):
        # small grids are bound by launch latency, where the per-launch
        # events of the timed region above add a large share: the same
        # number of further steps with only two events around them
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.step(dt, args.steps)
        e1.record(stream)
        e1.synchronize()
        no_events_ms = e0.elapsed_time(e1) / args.steps
    diag = ctx.diag()
    log(f"[bench] timed {args.steps} steps in {elapsed:.3f} s; diag {diag}")

    value = sweeps * cells * args.steps / elapsed
    # the dominant kernel: the sweep timing class with the largest share of
    # the step (at 48^3 x 48^3 the 256-pencil strided tiles: x2, x3 and both
    # v1 half-steps; the x1 sweep, which also sums the velocity moment, and
    # the two-axis v2/v3 pass of each kick are timed in classes of their
    # own); each class is one kernel instantiation moving 2 * es bytes per
    # cell per launch
    sweep_classes = ("sweep_strided_wide", "sweep_contiguous", "sweep_strided_other",
                     "sweep_x1_moment", "kick_plane")
    dom_name = max(sweep_classes, key=lambda k: tim[k]["total_ms"])
    dom = tim[dom_name]
    es = 4 if storage == slmpp.F32 else 8
    bytes_per_launch = 2.0 * es * cells
    avg_ms = dom["total_ms"] / max(dom["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    kernel_key = f"{spec['name']}/{args.dtype}"
    traffic = read_traffic(kernel_key)
    all_ms = sum(tim[k]["total_ms"] for k in sweep_classes)
    all_n = sum(tim[k]["launches"] for k in sweep_classes)
    per_class = {}
    for k, v in tim.items():
        if v["launches"]:
            avg = v["total_ms"] / v["launches"]
            per_class[k] = {"launches": v["launches"], "avg_ms": round(avg, 4),
                            "GB_s": round(v["bytes"] / v["launches"] / (avg * 1e-3) / 1e9, 1)}
            if v["cells"]:
                per_class[k]["cell_updates_per_s"] = v["cells"] / v["launches"] / (avg * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"{spec['name']} {spec['nx'][0]}^{D} x {spec['nv'][0]}^{D}, "
                        f"SL-MPP{spec['order']}, {args.dtype} f, fp64 moment+Poisson",
            "cells": cells,
            "sweeps_per_step": sweeps,
            "dt": dt,
            "f_placement": placement,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": ("kick_plane_kernel" if dom_name == "kick_plane" else "sweep_fast_kernel")
                      + f", timing class {dom_name}",
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": round(avg_ms, 4),
            "launches": dom["launches"],
            "all_sweeps_GB_s": round(bytes_per_launch * all_n / (all_ms * 1e-3) / 1e9, 1),
        },
        "detail": {"per_class": per_class, "mass": diag["mass"], "f_min": diag["f_min"],
                   "nonfinite": diag["nonfinite"]},
    }
    if no_events_ms is not None:
        out["detail"]["without_launch_events"] = {
            "steps": args.steps, "ms_per_step": no_events_ms,
            "cell_updates_per_s": sweeps * cells / (no_events_ms * 1e-3)}
    # velocity-space diagnostics of the same f (each one read of f)
    nxs = int(np.prod(spec["nx"][:D]))
    nvs = int(np.prod(spec["nv"][:D]))
    rho_d = torch.empty(nxs, dtype=torch.float64, device=dev)
    mean_d = torch.empty(D * nxs, dtype=torch.float64, device=dev)
    disp_d = torch.empty(D * nxs, dtype=torch.float64, device=dev)
    F_d = torch.empty(nvs, dtype=torch.float64, device=dev)
    es_f = 4 if storage == slmpp.F32 else 8
    diag_rates = {}
    for name, fn in (("density_moment", lambda: ctx.density_moment(rho_d)),
                     ("velocity_moments", lambda: ctx.velocity_moments(rho_d, mean_d, disp_d)),
                     ("velocity_distribution", lambda: ctx.velocity_distribution(F_d))):
        fn()
        ctx.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            fn()
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 3
        diag_rates[name] = {"ms": round(ms, 3), "GB_s": round(es_f * cells / (ms * 1e-3) / 1e9, 1)}
    out["detail"]["diagnostics"] = diag_rates
    log(f"[bench] diagnostics: {diag_rates}")
    del rho_d, mean_d, disp_d, F_d

    if args.fp64_compare > 0 and storage == slmpp.F32:
        # the same workload from the same start with FP64 storage on the same
        # GPU: its rate, and the error of FP32 storage after the same steps
        total = args.warmup + args.steps
        f64_buf, f64_t, _ = alloc_f(slmpp, torch, fshape, torch.float64, dev)
        ctx64 = slmpp.Context(slmpp.make_desc(spec, slmpp.F64), f=f64_t, stream=stream, device=dev)
        ctx64.init_f_separable(s, gv)
        ctx64.field()
        d64_0 = ctx64.diag()
        ctx64.step(dt, 1)
        ctx64.sync()
        n64 = max(total - 1, 1)
        t0 = time.perf_counter()
        ctx64.step(dt, n64)
        ctx64.sync()
        e64 = time.perf_counter() - t0
        d64 = ctx64.diag()
        num = torch.zeros((), dtype=torch.float64, device=dev)
        den = torch.zeros((), dtype=torch.float64, device=dev)
        a32 = ctx.f.reshape(-1)
        a64 = ctx64.f.reshape(-1)
        chunk = 1 << 27
        with torch.cuda.stream(stream):
            for c0 in range(0, cells, chunk):
                x = a32[c0:c0 + chunk].double()
                y = a64[c0:c0 + chunk]
                num += (x - y).abs().sum()
                den += y.abs().sum()
                del x
        stream.synchronize()
        out["detail"]["fp64_same_workload"] = {
            "steps": n64,
            "cell_updates_per_s": sweeps * cells * n64 / e64,
            "ms_per_step": e64 / n64 * 1e3,
        }
        out["detail"]["fp32_vs_fp64"] = {
            "steps": total,
            "l1_rel": (num / den).item(),
            "mass_drift_f32": abs(diag["mass"] - diag0["mass"]) / abs(diag0["mass"]),
            "mass_drift_f64": abs(d64["mass"] - d64_0["mass"]) / abs(d64_0["mass"]),
            "field_energy_rel_diff": abs(diag["field_energy"] - d64["field_energy"]) / abs(d64["field_energy"]),
            "mode_amp_rel_diff": abs(diag["mode_amp"] - d64["mode_amp"]) / abs(d64["mode_amp"]),
        }
        log(f"[bench] fp32 vs fp64 after {total} steps: {out['detail']['fp32_vs_fp64']}")
        del a32, a64
        ctx64.close()
        del ctx64, f64_t
        release_f(torch, f64_buf)
    ctx.close()
    del ctx, f_t
    release_f(torch, f_buf)
    torch.cuda.empty_cache()

    if args.merge_compare > 0:
        # the same workload with merged velocity half-steps (6 instead of 9
        # sweeps per step for 3D3V within a call)
        sp = dict(spec, merge_kicks=True)
        c = slmpp.Context(slmpp.make_desc(sp, storage), stream=stream, device=dev)
        c.init_f_separable(s, gv)
        c.field()
        c.step(dt, 1)
        c.sync()
        t0 = time.perf_counter()
        c.step(dt, args.merge_compare)
        c.sync()
        em = (time.perf_counter() - t0) / args.merge_compare * 1e3
        out["detail"]["merged_kicks"] = {"steps_per_call": args.merge_compare,
                                         "ms_per_step": round(em, 2),
                                         "sweeps_per_step": 2 * D,
                                         "step_speedup": round(out["ms_per_step"] / em, 3)}
        log(f"[bench] merged kicks: {out['detail']['merged_kicks']}")
        c.close()
        del c
        torch.cuda.empty_cache()

    if args.rk_compare > 0 and args.workload == "landau_3d3v":
        # the paper's cost comparison (Sec. 4): RK-MPP5 against SL-MPP5 on the
        # same 48^3 x 48^3 workload and storage (x-CFL 0.2 suits both)
        rk = {}
        for scheme in ("sl", "rk3"):
            sp = W.landau_3d3v(n=48, order=5)
            sp["time"] = scheme
            c = slmpp.Context(slmpp.make_desc(sp, storage), stream=stream, device=dev)
            c.init_f_separable(*W.separable_factors(sp))
            c.field()
            c.step(sp["dt"], 1)
            c.sync()
            t0 = time.perf_counter()
            c.step(sp["dt"], args.rk_compare)
            c.sync()
            rk[scheme] = (time.perf_counter() - t0) / args.rk_compare * 1e3
            c.close()
            del c
            torch.cuda.empty_cache()
        out["detail"]["rk_mpp5_vs_sl_mpp5"] = {
            "workload": "landau_3d3v 48^3 x 48^3, order 5, same dt", "steps": args.rk_compare,
            "sl_mpp5_ms_per_step": round(rk["sl"], 2), "rk_mpp5_ms_per_step": round(rk["rk3"], 2),
            "rk_over_sl": round(rk["rk3"] / rk["sl"], 3)}
        log(f"[bench] RK-MPP5 vs SL-MPP5: {out['detail']['rk_mpp5_vs_sl_mpp5']}")

    if args.ensemble_steps > 0 and storage == slmpp.F32:
        out["detail"]["ensemble"] = ensemble_leg(args.ensemble_steps, 5, "f32", compare_fp64=True)
        torch.cuda.empty_cache()

    # reference: a plain streaming copy of 4 GiB with the library's copy kernel
    nbytes = 4 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    with torch.cuda.stream(stream):
        slmpp.copy_device(dst.data_ptr(), src.data_ptr(), nbytes, stream)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(5):
            slmpp.copy_device(dst.data_ptr(), src.data_ptr(), nbytes, stream)
        ev1.record(stream)
    ev1.synchronize()
    out["detail"]["copy_kernel_GBs"] = round(5 * 2 * nbytes / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline at {args.cpu_sample}^{D} and {args.cpu_sample_1t}^{D}")

        def spec_fn(n):
            if args.workload == "landau_3d3v":
                return W.landau_3d3v(n=n, order=7)
            if args.workload == "jeans_3d3v":
                return W.jeans_3d3v(n=n, order=5)
            if args.workload == "collapse_3d3v":
                return W.collapse_3d3v(nx=n, nv=n // 2, order=5)
            return workload(args.workload, args.dtype)

        out["cpu_baseline"] = cpu_baseline(spec_fn, args.cpu_sample, args.cpu_sample_1t)
    print(json.dumps(out), flush=True)


def ensemble_main(args):
    """--workload ensemble: the batched form as the bench line."""
    from paper_1702_08521_amd import workloads as W

    ens = ensemble_leg(args.steps, args.warmup, args.dtype, compare_fp64=args.fp64_compare > 0)
    es = 4 if args.dtype == "f32" else 8
    achieved = ens["step_bytes"] / (ens["graph_ms_per_step"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": ens["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ens["graph_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"ensemble of {ens['runs']} Landau-type runs (1D1V and 2D2V, "
                               f"SL-MPP5/7 mixed, seed {W.ENSEMBLE_SEED}), "
                               f"{args.dtype} f, graph-captured step",
                   "cells": ens["cells"], "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole captured step (batch tables, sweep and two-axis kick "
                               "passes, moment, Poisson)",
                     "bytes_per_step": ens["step_bytes"], "element_bytes": es},
        "detail": ens,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = ensemble_cpu_baseline(W.ensemble(), args.cpu_steps)
    print(json.dumps(out), flush=True)


def ensemble_cpu_baseline(specs, steps):
    """FP64 oracle: `steps` Strang steps of every run of the ensemble."""
    import numpy as np

    import oracle as O

    O.use_native()
    runs = [O.Run(s) for s in specs]
    t0 = time.perf_counter()
    for run, s in zip(runs, specs):
        run.step(s["dt"], steps)
    dt = time.perf_counter() - t0
    upd = steps * sum(int(np.prod(s["nx"][:s["D"]])) * int(np.prod(s["nv"][:s["D"]])) * 3 * s["D"]
                      for s in specs)
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    return {"value": upd / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": (f"{steps} Strang steps of all {len(specs)} ensemble runs, FP64 oracle, gcc -O3 "
                       f"-march=native -ffp-contract=off, OpenMP over pencils, on {cpu_model()} "
                       f"({threads} threads), {dt:.2f} s")}


if __name__ == "__main__":
    main()
