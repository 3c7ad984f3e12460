"""Benchmark of the MFA evaluator / ray caster on one MI355X.

One step = the whole hot path over one batch of the 128^3 workload: a
single block of 128^3 FP32 control points (degree 3, clamped uniform knots,
64-Gaussian field), decoded for value + gradient on a 512^3 parameter grid
and at 10^7 uniform random points, plus one 1024x1024 perspective frame
(up to 1024 samples per ray, transfer function, Phong, early termination).
The random points are decoded through the library's block/tile sort (the
sort is inside the timed step).  Inputs are resident in device memory
before timing starts.

Prints one JSON line.  value = decoded samples (value + gradient) per second
over the step, counting the grid points, the random points and the frame
samples whose value and gradient the renderer evaluates.  Samples that the
renderer steps over exactly (the transfer function is zero over the value
bounds of their cell, so they cannot change the pixel) are not decoded and
not counted; they are reported as frame_samples_stepped.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "decoded samples/s (value+grad), ms/frame at 1024², p50/p99 request latency"

# algorithmic work per unit (degree 3): value + gradient sample, render sample
FLOP_SAMPLE_P3 = 504
FLOP_RENDER_SAMPLE_P3 = 558
PEAK_FP32_TFLOPS = 157.3           # published FP32 vector peak (packed FMA)
PEAK_FP32_ISSUABLE_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 flop x 2.4 GHz, unpacked FMA
PEAK_HBM_GBS = 8000.0

GRID_N = 512
N_POINTS = 10_000_000
FRAME = 1024

# HBM bytes per launch of a kernel of the default workload (FP32 storage),
# from rocprofv3 --pmc runs of this script, one counter per run (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
# reads on the plain copy that --copy-calibration adds (bytes moved / KiB
# read).  An entry holds only for the kernel source it was measured on.
TRAFFIC = {
    # 1024^2 frame of the 128^3 model; copy reference: 512 MiB read + 512 MiB
    # written, FETCH_SIZE 262161 KiB (scale 2.0), WRITE_SIZE 524288 KiB (1.0)
    "render": {"kernels_sha256": "456ff8e1afe37b889a77c650fcbf70f3db4e28e349da79b8d7f68bebbac1b542",
               "fetch_kib": 35984.4, "fetch_scale": 2.0, "write_kib": 16396.7, "write_scale": 1.0},
}


def kernel_source_sha256() -> str:
    import hashlib
    path = os.path.join(ROOT, "paper_2312_15073_amd", "csrc", "mfa_kernels.hip")
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def traffic_bytes(kernel: str, storage: str):
    t = TRAFFIC.get(kernel)
    if t is None or storage != "f32" or t["kernels_sha256"] != kernel_source_sha256():
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def flop_per_sample(p: int) -> int:
    q = p + 1
    return 2 * (2 * q ** 3 + 3 * q ** 2 + 4 * q) + 6 * (q * p + q * (p - 1))


# ------------------------------------------------------------------ CPU baseline (oracle)
def _cpu_job(job):
    from oracle import bspline as ob
    from oracle import render as orr
    kind, arg = job
    spec = _CPU_STATE["spec"]
    if kind == "grid":
        ax = _CPU_STATE["axis"]
        a0, a1 = arg
        ob.decode_grid(spec, [ax[a0:a1], ax, ax])
        return (a1 - a0) * len(ax) * len(ax)
    if kind == "points":
        ob.evaluate(spec, arg.T.astype(np.float64))
        return arg.shape[1]
    cam, params, pix = arg
    r = orr.render(orr.model_field(spec), spec.lo, spec.hi, cam, params, FRAME, FRAME, pixels=pix)
    return int(r["used"].sum())


_CPU_STATE = {}


def cpu_baseline(spec, cam, params, pts):
    """The FP64 oracle on 1/64 of each component of the step, over the host
    cores (fork pool started before any GPU use)."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    _CPU_STATE["spec"] = spec
    _CPU_STATE["axis"] = synth.grid_axis(GRID_N)
    jobs = []
    planes = GRID_N // 64                           # 8 of 512 planes
    p0 = GRID_N // 2 - planes // 2
    for a in range(p0, p0 + planes):
        jobs.append(("grid", (a, a + 1)))
    sub = pts[:, : N_POINTS // 64]
    for c in np.array_split(np.arange(sub.shape[1]), cores):
        jobs.append(("points", np.ascontiguousarray(sub[:, c])))
    crop = FRAME // 8                               # 128x128 = 1/64 of the pixels
    r0 = FRAME // 2 - crop // 2
    rows = np.arange(r0, r0 + crop)
    for rr in np.array_split(rows, 4 * cores):
        pix = np.stack(np.meshgrid(rr, np.arange(r0, r0 + crop), indexing="ij"), -1).reshape(-1, 2)
        jobs.append(("render", (cam, params, pix)))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        counts = pool.map(_cpu_job, jobs, chunksize=1)
    dt = time.perf_counter() - t0
    n = int(sum(counts))
    return {"value": n / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 NumPy oracle on 1/64 of the step: {planes} of {GRID_N} grid planes, "
                       f"{sub.shape[1]} of {N_POINTS} points, the central {crop}x{crop} pixels of "
                       f"the {FRAME}x{FRAME} frame; {n} samples in {dt:.1f} s"),
            "cpu_model": _cpu_model()}


def _cpu_model() -> str:
    """The host CPU as lscpu names it (model name, family/model/stepping,
    sockets x cores x threads, hypervisor), else /proc/cpuinfo's model name."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                             text=True, timeout=10).stdout
        f = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f[k.strip()] = v.strip()
        if "Model name" in f:
            desc = f["Model name"]
            if "CPU family" in f:
                desc += (f" (family {f['CPU family']}, model {f.get('Model', '?')}, "
                         f"stepping {f.get('Stepping', '?')})")
            desc += (f"; {f.get('Socket(s)', '?')} socket(s) x {f.get('Core(s) per socket', '?')} "
                     f"cores x {f.get('Thread(s) per core', '?')} threads, {f.get('CPU(s)', '?')} CPUs")
            if "Hypervisor vendor" in f:
                desc += f", {f['Hypervisor vendor']} guest"
            return desc
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ------------------------------------------------------------------ GPU run
def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="single128",
                    choices=["single128", "multiblock", "serving", "points", "encode", "encode_adaptive",
                             "composite", "iso", "graded", "quality", "storage", "values", "cr_sweep"],
                    help="single128: 128^3 model, 512^3 grid + 1e7 points + 1024^2 frame (default); "
                         "multiblock: 8x8x8 blocks, 1e8 sorted points + 2048^2 frame; "
                         "serving: open-loop request trace over three resident models; "
                         "points: point decode alone, input order vs block/tile-sorted order; "
                         "encode: least-squares fit of a 512^3 sample grid to 192^3 control points; "
                         "encode_adaptive: the 512^3 grid fitted with knot insertion to 1e-4; "
                         "quality: Marschner-Lobb frames, MFA vs local filters, PSNR vs analytic; "
                         "graded: the default step on the 128^3 model with graded knots; "
                         "iso: first-hit isosurface of the 128^3 model's 1024^2 frame; "
                         "composite: 8 octant partial renders of the 8x8x8-block frame + over; "
                         "storage: FP32 vs BF16 vs FP16 storage on the 128^3 and 8x8x8-block steps, "
                         "kernel times and image error against the FP64 oracle and the analytic "
                         "field; values: value-only vs value+gradient queries (grid and points); "
                         "cr_sweep: Marschner-Lobb 256^3 encoded at compression ratios 20..212, "
                         "encode time, ms/frame and PSNR")
    ap.add_argument("--storage-model", default="both", choices=["both", "single128", "multiblock"],
                    help="storage: which model(s) to compare")
    ap.add_argument("--points-model", default="single128", choices=["single128", "multiblock"],
                    help="points: the 128^3 model with 1e7 points or the 8x8x8-block model with 1e8")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run two plain device copies of this many MiB before timing (reference "
                         "for HBM byte counters)")
    ap.add_argument("--requests", type=int, default=10000, help="serving: measured requests")
    ap.add_argument("--batch-items", type=int, default=4096, help="serving: work items per batch")
    ap.add_argument("--load", type=float, default=0.6, help="serving: offered load / capacity")
    args = ap.parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU path is a design, not part of this build", file=sys.stderr)
        return 2
    if args.workload == "multiblock":
        return run_multiblock(args)
    if args.workload == "serving":
        return run_serving(args)
    if args.workload == "points":
        return run_points(args)
    if args.workload == "encode":
        return run_encode(args)
    if args.workload == "encode_adaptive":
        return run_encode_adaptive(args)
    if args.workload == "composite":
        return run_composite(args)
    if args.workload == "iso":
        return run_iso(args)
    if args.workload == "quality":
        return run_quality(args)
    if args.workload == "storage":
        return run_storage(args)
    if args.workload == "values":
        return run_values(args)
    if args.workload == "cr_sweep":
        return run_cr_sweep(args)
    if args.workload == "graded":
        if args.steps is None:
            args.steps = 20
        return run_single128(args, graded=True)
    if args.steps is None:
        args.steps = 20
    return run_single128(args)


def run_single128(args, graded: bool = False):
    spec = synth.model_c2_graded() if graded else synth.model_c2()
    p = spec.blocks[0].degree[0]
    pts = synth.random_points(N_POINTS, seed=12)
    cam = synth.perspective_camera(FRAME, FRAME)
    params = synth.render_params(spec)
    cpu = None if args.no_cpu_baseline else cpu_baseline(spec, cam, params, pts)

    import torch
    import paper_2312_15073_amd as mfa

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    copy_calibration(torch, dev, args.copy_calibration)
    model = mfa.Model(spec, args.storage)
    axes = [torch.as_tensor(synth.grid_axis(GRID_N), device=dev) for _ in range(3)]
    xyz = torch.as_tensor(pts, device=dev)
    tf = torch.as_tensor(params["tf"], device=dev)
    grid_out = torch.empty((GRID_N, GRID_N, GRID_N, 4), dtype=torch.float32, device=dev)
    pts_out = torch.empty((N_POINTS, 4), dtype=torch.float32, device=dev)
    rgba = torch.empty((FRAME, FRAME, 4), dtype=torch.float32, device=dev)

    # samples the frame composites (exact, from the kernel's own counters)
    _, ns, ne = mfa.render_frame(model, cam, params, FRAME, FRAME, tf_dev=tf, nsamp=True,
                                 neval=True, device=dev)
    torch.cuda.synchronize()
    s_frame = int(ns[..., 1].sum().item())
    s_eval = int(ne.sum().item())
    del ns, ne
    n_grid = GRID_N ** 3
    samples_step = n_grid + N_POINTS + s_eval       # decoded samples only

    names = ["decode_grid", "decode_points", "render"]

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        mfa.decode_grid(model, axes, out=grid_out)
        if ev is not None:
            ev[1].record(stream)
        mfa.decode_points(model, xyz, out=pts_out, sorted_order=True)
        if ev is not None:
            ev[2].record(stream)
        mfa.render_frame(model, cam, params, FRAME, FRAME, tf_dev=tf, out=rgba, device=dev)
        if ev is not None:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms = {n: float(np.mean([events[k][i].elapsed_time(events[k][i + 1])
                                 for k in range(args.steps)])) for i, n in enumerate(names)}
    ms_step = 1e3 * elapsed / args.steps
    info = model.info()

    fl = flop_per_sample(p)
    fl_r = fl + 54
    model_bytes = info["ctrl_bytes"]     # the model read once per launch (device_bytes also
                                         # counts the sorted decode's scratch)
    grid_bytes = n_grid * 16 + model_bytes + 3 * GRID_N * 8
    pts_bytes = N_POINTS * 28 + model_bytes
    kernels = {
        "decode_grid": dict(ms=kern_ms["decode_grid"], samples=n_grid, bound="hbm",
                            achieved=grid_bytes / kern_ms["decode_grid"] / 1e6, unit="GB/s",
                            peak=PEAK_HBM_GBS, bytes_per_launch=grid_bytes),
        "decode_points": dict(ms=kern_ms["decode_points"], samples=N_POINTS, bound="hbm",
                              achieved=pts_bytes / kern_ms["decode_points"] / 1e6, unit="GB/s",
                              peak=PEAK_HBM_GBS, bytes_per_launch=pts_bytes,
                              tflops=N_POINTS * fl / kern_ms["decode_points"] / 1e9),
        # algorithmic work of a frame: full value+gradient+shading work for the
        # samples evaluated; samples skipped as transparent count no flops
        "render": dict(ms=kern_ms["render"], samples=s_frame, evaluated_samples=s_eval,
                       bound="alu", achieved=s_eval * fl_r / kern_ms["render"] / 1e9,
                       unit="TFLOP/s", peak=PEAK_FP32_TFLOPS, flop_per_launch=s_eval * fl_r),
    }
    for k in kernels.values():
        k["frac"] = k["achieved"] / k["peak"]
        k["samples_per_s"] = k["samples"] / (k["ms"] * 1e-3)
    dom = max(kernels, key=lambda n: kernels[n]["ms"])
    dk = kernels[dom]
    roofline = {"bound": dk["bound"], "achieved": dk["achieved"], "peak": dk["peak"],
                "unit": dk["unit"], "frac": dk["frac"],
                "traffic": traffic_bytes(dom, args.storage), "kernel": dom}
    if dk["bound"] == "alu":
        roofline["peak_unpacked_fp32"] = PEAK_FP32_ISSUABLE_TFLOPS
        roofline["frac_unpacked_fp32"] = dk["achieved"] / PEAK_FP32_ISSUABLE_TFLOPS
    line = {
        "metric": METRIC,
        "value": samples_step / (ms_step * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"f32 ({args.storage} storage)",
        "data": "synthetic",
        "config": {"workload": (f"single block, {spec.blocks[0].ctrl.shape[0]}^3 control points"
                                f"{' on graded knots (span widths 7x apart)' if graded else ''}, "
                                f"degree {p}, {args.storage} storage; decode {GRID_N}^3 grid + "
                                f"{N_POINTS} random points + {FRAME}x{FRAME} perspective frame "
                                f"(max 1024 samples/ray)"),
                   "samples_per_step": samples_step, "frame_samples": s_frame,
                   "frame_samples_evaluated": s_eval, "frame_samples_stepped": s_frame - s_eval,
                   "parallelism": "single GPU"},
        "ms_per_frame": kern_ms["render"],
        "kernels": kernels,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    model.close()
    return 0


# ------------------------------------------------------------------ 8x8x8-block workload
MB_POINTS = 100_000_000
MB_FRAME = 2048


def _cpu_job_mb(job):
    from oracle import bspline as ob
    from oracle import render as orr
    kind, arg = job
    spec = _CPU_STATE["spec"]
    if kind == "points":
        ob.evaluate(spec, arg.T.astype(np.float64))
        return arg.shape[1]
    cam, params, pix = arg
    r = orr.render(orr.model_field(spec), spec.lo, spec.hi, cam, params, MB_FRAME, MB_FRAME, pixels=pix)
    return int(r["used"].sum())


def cpu_baseline_mb(spec, cam, params, pts):
    """The FP64 oracle on 2e5 of the points and the central 96x96 pixels."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    _CPU_STATE["spec"] = spec
    sub = pts[:, :200_000]
    jobs = [("points", np.ascontiguousarray(sub[:, c]))
            for c in np.array_split(np.arange(sub.shape[1]), cores)]
    crop = 96
    r0 = MB_FRAME // 2 - crop // 2
    for rr in np.array_split(np.arange(r0, r0 + crop), 4 * cores):
        pix = np.stack(np.meshgrid(rr, np.arange(r0, r0 + crop), indexing="ij"), -1).reshape(-1, 2)
        jobs.append(("render", (cam, params, pix)))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        n = int(sum(pool.map(_cpu_job_mb, jobs, chunksize=1)))
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": (f"FP64 NumPy oracle: {sub.shape[1]} of {MB_POINTS} points and the central "
                       f"{crop}x{crop} pixels of the {MB_FRAME}^2 frame; {n} samples in {dt:.1f} s"),
            "cpu_model": _cpu_model()}


def run_multiblock(args):
    """Step = block/tile-sorted decode of 1e8 points + one 2048^2 frame of the
    8x8x8-block model (~57M control points, degree 3)."""
    steps = 5 if args.steps is None else args.steps
    spec = synth.model_c4()
    pts = synth.random_points(MB_POINTS, seed=14)
    cam = synth.perspective_camera(MB_FRAME, MB_FRAME)
    params = synth.render_params(spec, max_samples=2048)
    cpu = None if args.no_cpu_baseline else cpu_baseline_mb(spec, cam, params, pts)
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    model = mfa.Model(spec, args.storage)
    xyz = torch.as_tensor(pts, device=dev)
    del pts
    tf = torch.as_tensor(params["tf"], device=dev)
    pts_out = torch.empty((MB_POINTS, 4), dtype=torch.float32, device=dev)
    rgba = torch.empty((MB_FRAME, MB_FRAME, 4), dtype=torch.float32, device=dev)
    _, ns, ne = mfa.render_frame(model, cam, params, MB_FRAME, MB_FRAME, tf_dev=tf, nsamp=True,
                                 neval=True, device=dev)
    torch.cuda.synchronize()
    s_frame, s_eval = int(ns[..., 1].sum().item()), int(ne.sum().item())
    del ns, ne

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        mfa.decode_points(model, xyz, out=pts_out, sorted_order=True)
        if ev:
            ev[1].record(stream)
        mfa.render_frame(model, cam, params, MB_FRAME, MB_FRAME, tf_dev=tf, out=rgba, device=dev)
        if ev:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(events[k])
    torch.cuda.synchronize()
    ms_step = 1e3 * (time.perf_counter() - t0) / steps
    kms = {n: float(np.mean([events[k][i].elapsed_time(events[k][i + 1]) for k in range(steps)]))
           for i, n in enumerate(["decode_points", "render"])}
    info = model.info()
    fl_r = flop_per_sample(3) + 54
    kernels = {
        "decode_points": dict(ms=kms["decode_points"], samples=MB_POINTS, bound="hbm",
                              achieved=(MB_POINTS * 28 + info["ctrl_bytes"]) / kms["decode_points"] / 1e6,
                              unit="GB/s", peak=PEAK_HBM_GBS),
        "render": dict(ms=kms["render"], samples=s_frame, evaluated_samples=s_eval, bound="alu",
                       achieved=s_eval * fl_r / kms["render"] / 1e9, unit="TFLOP/s",
                       peak=PEAK_FP32_TFLOPS),
    }
    for k in kernels.values():
        k["frac"] = k["achieved"] / k["peak"]
        k["samples_per_s"] = k["samples"] / (k["ms"] * 1e-3)
    dom = max(kernels, key=lambda n: kernels[n]["ms"])
    dk = kernels[dom]
    roofline = {"bound": dk["bound"], "achieved": dk["achieved"], "peak": dk["peak"],
                "unit": dk["unit"], "frac": dk["frac"], "traffic": None, "kernel": dom}
    samples_step = MB_POINTS + s_eval                # decoded samples only
    print(json.dumps({
        "metric": METRIC, "value": samples_step / (ms_step * 1e-3), "unit": "samples/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"f32 ({args.storage} storage)",
        "data": "synthetic",
        "config": {"workload": (f"8x8x8 blocks, {info['n_ctrl_total']} control points (24..72 per "
                                f"axis and block), degree 3, {args.storage} storage; block/tile-"
                                f"sorted decode of {MB_POINTS} random points + {MB_FRAME}^2 "
                                f"perspective frame (max 2048 samples/ray)"),
                   "samples_per_step": samples_step, "frame_samples": s_frame,
                   "frame_samples_evaluated": s_eval, "frame_samples_stepped": s_frame - s_eval,
                   "parallelism": "single GPU"},
        "ms_per_frame": kms["render"], "kernels": kernels, "roofline": roofline,
        "cpu_baseline": cpu}), flush=True)
    model.close()
    return 0


def copy_calibration(torch, dev, mib):
    """Two plain device-to-device copies of `mib` MiB: the reference the HBM
    byte counters (FETCH_SIZE, WRITE_SIZE) are scaled by."""
    if mib <= 0:
        return
    a = torch.ones(mib * 2 ** 18, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


# ------------------------------------------------------------------ point-decode workload
def run_points(args):
    """Point decode alone: the same points in input order and through the
    block/tile sort, timed per call with HIP events."""
    steps = 5 if args.steps is None else args.steps
    if args.points_model == "multiblock":
        spec, n, seed, name = synth.model_c4(), MB_POINTS, 14, "8x8x8-block model"
    else:
        spec, n, seed, name = synth.model_c2(), N_POINTS, 12, "single block, 128^3 control points"
    pts = synth.random_points(n, seed=seed)
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    copy_calibration(torch, dev, args.copy_calibration)
    model = mfa.Model(spec, args.storage)
    xyz = torch.as_tensor(pts, device=dev)
    del pts
    out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    res = {}
    for label, srt in (("input_order", False), ("sorted", True)):
        for _ in range(args.warmup):
            mfa.decode_points(model, xyz, out=out, sorted_order=srt)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for k in range(steps):
            mfa.decode_points(model, xyz, out=out, sorted_order=srt)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))
        res[label] = {"ms": ms, "samples_per_s": n / (ms * 1e-3)}
    info = model.info()
    print(json.dumps({
        "metric": "decoded samples/s (value+grad), random points", "value": res["sorted"]["samples_per_s"],
        "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": res["sorted"]["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.storage == "f32" else f"f32 ({args.storage} storage)",
        "data": "synthetic",
        "config": {"workload": f"{name} ({info['n_ctrl_total']} control points, degree 3, "
                               f"{args.storage} storage), {n} uniform random points",
                   "parallelism": "single GPU"},
        "decode": res, "sorted_speedup": res["input_order"]["ms"] / res["sorted"]["ms"]}), flush=True)
    model.close()
    return 0


# ------------------------------------------------------------------ encode workload
ENC_RES, ENC_CTRL, ENC_P = 512, 192, 3      # 512^3 samples -> 192^3 control points (CR 18.96)


def encode_flop(res, n_ctrl) -> float:
    """Multiply-add count x 2 of the three mode products."""
    N0, N1, N2 = res
    n0, n1, n2 = n_ctrl
    return 2.0 * (n0 * N0 * N1 * N2 + n1 * N1 * n0 * N2 + n2 * N2 * n0 * n1)


def _encode_bytes(res, n_ctrl) -> float:
    """Algorithmic bytes of one apply: the FP32 samples read once, the two
    FP64 intermediate products written and read once, the FP64 control
    points written, the three FP64 pseudo-inverse tables read."""
    N0, N1, N2 = res
    n0, n1, n2 = n_ctrl
    return (4.0 * N0 * N1 * N2 + 16.0 * n0 * N1 * N2 + 16.0 * n0 * n1 * N2 + 8.0 * n0 * n1 * n2
            + 8.0 * (n0 * N0 + n1 * N1 + n2 * N2))


def _encode_cpu_baseline():
    """The oracle's fit of a 256^3 block of the same field to 96^3 control
    points (the same compression ratio), repeated for at least 3 s on the
    host."""
    from oracle import encode as oe
    field = synth.field_c2()
    xs = np.arange(256, dtype=np.float64) / 255
    F = field.value_separable(xs, xs, xs).astype(np.float32).astype(np.float64)
    T = synth.clamped_uniform_knots(96, ENC_P)
    reps, t0 = 0, time.perf_counter()
    while True:
        oe.fit_grid(F, [xs] * 3, [ENC_P] * 3, [T] * 3, [96] * 3)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= 3.0:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": reps * 256 ** 3 / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 NumPy oracle fit of a 256^3 block to 96^3 control points, {reps} fits "
                      f"in {dt:.1f} s (BLAS threads: {threads})", "cpu_model": _cpu_model()}


def _field_c2_samples(N: int, dev):
    """FP32 samples (N, N, N) of the 64-Gaussian field on the uniform grid,
    made on the GPU."""
    import torch
    field = synth.field_c2()
    xs = torch.arange(N, dtype=torch.float64, device=dev) / (N - 1)
    F = torch.zeros((N, N, N), dtype=torch.float64, device=dev)
    for c, sg, a in zip(field.centres, field.sigmas, field.amps):
        e = [torch.exp(-(xs - float(c[q])) ** 2 / (2.0 * float(sg) ** 2)) for q in range(3)]
        F += float(a) * e[0][:, None, None] * e[1][None, :, None] * e[2][None, None, :]
    return F.to(torch.float32).contiguous()


def recon_flop(res, n_ctrl) -> float:
    """Multiply-add count x 2 of the three mode products that take control
    points back to the sample grid."""
    N0, N1, N2 = res
    n0, n1, n2 = n_ctrl
    return 2.0 * (N0 * n0 * n1 * n2 + N1 * n1 * N0 * n2 + N2 * n2 * N0 * N1)


ADA_INIT, ADA_EMAX, ADA_CAP, ADA_FITS = 32, 1e-4, 256, 12


def _encode_adaptive_cpu_baseline():
    """The oracle's adaptive fit of a 128^3 grid of the same field (same
    initial knots and bound, cap 128), repeated for at least 3 s."""
    from oracle import encode as oe
    field = synth.field_c2()
    xs = np.arange(128, dtype=np.float64) / 127
    F = field.value_separable(xs, xs, xs).astype(np.float32).astype(np.float64)
    reps, t0 = 0, time.perf_counter()
    while True:
        _, _, hist = oe.fit_adaptive(F, [xs] * 3, [ENC_P] * 3, [ADA_INIT] * 3, ADA_EMAX,
                                     max_iter=ADA_FITS, max_ctrl=[min(ADA_CAP, 128)] * 3)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= 3.0:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": reps * 128 ** 3 / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 NumPy oracle adaptive fit of a 128^3 grid from {ADA_INIT}^3 control points "
                      f"({len(hist)} fits, final {hist[-1][0]}), {reps} runs in {dt:.1f} s "
                      f"(BLAS threads: {threads})", "cpu_model": _cpu_model()}


def run_encode_adaptive(args):
    """Encoding with knot insertion of the 512^3 FP32 grid of the 64-Gaussian
    field: from 32^3 clamped uniform control points, fits and knot halving
    until every span's largest relative error is below 1e-4 (at most 256
    control points per axis, 12 fits).  One step = the whole adaptive call,
    host split decisions included."""
    steps = 5 if args.steps is None else args.steps
    cpu = None if args.no_cpu_baseline else _encode_adaptive_cpu_baseline()
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N = ENC_RES
    values = _field_c2_samples(N, dev)
    axis = [np.arange(N, dtype=np.float64) / (N - 1)] * 3
    cap = (ADA_CAP,) * 3
    work = torch.empty((mfa.encode_adaptive_workspace_bytes((N,) * 3, cap),), dtype=torch.uint8,
                       device=dev)

    def step():
        return mfa.encode_adaptive(values, axis, (ENC_P,) * 3, (ADA_INIT,) * 3, ADA_EMAX,
                                   max_ctrl=cap, max_fits=ADA_FITS, work=work)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        knots, P, hist = step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    flop = sum(encode_flop((N,) * 3, h[0]) + recon_flop((N,) * 3, h[0]) for h in hist)
    tf = flop / (ms * 1e-3) / 1e12
    print(json.dumps({
        "metric": "encoded samples/s (least-squares fit with knot insertion)",
        "value": N ** 3 / (ms * 1e-3), "unit": "samples/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (f32 samples)", "data": "synthetic",
        "config": {"workload": f"{N}^3 FP32 samples of the 64-Gaussian field, degree {ENC_P}, "
                               f"knot insertion from {ADA_INIT}^3 control points to relative error "
                               f"{ADA_EMAX} (cap {ADA_CAP} per axis, {ADA_FITS} fits)",
                   "fits": [[list(h[0]), h[1]] for h in hist], "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": tf, "peak": 78.6, "unit": "TFLOP/s",
                     "frac": tf / 78.6, "traffic": None,
                     "kernel": "whole call (fit + reconstruction GEMMs of every pass over the "
                               "call's wall time, error scans and host decisions included)",
                     "flop_per_launch": flop},
        "cpu_baseline": cpu}), flush=True)
    return 0


def run_encode(args):
    """Fixed-knot least-squares encoding of a 512^3 FP32 sample grid of the
    64-Gaussian field to 192^3 control points (degree 3): one plan, then
    timed applies (axis 0 by the banded route: B0^T F and the two banded
    solves per fiber; axes 1 and 2 as FP64 GEMMs on the matrix cores).  The
    roofline is by bytes: each product reads its input once and writes its
    output once (the axis-0 route's intermediate y is counted too, it goes
    through memory)."""
    steps = 10 if args.steps is None else args.steps
    cpu = None if args.no_cpu_baseline else _encode_cpu_baseline()
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    N, n = ENC_RES, ENC_CTRL
    values = _field_c2_samples(N, dev)
    axis = np.arange(N, dtype=np.float64) / (N - 1)
    t0 = time.perf_counter()
    plan = mfa.EncodePlan((N, N, N), [axis] * 3, (ENC_P,) * 3, (n, n, n), device=dev)
    plan_ms = 1e3 * (time.perf_counter() - t0)
    out = torch.empty((n, n, n), dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        plan.apply(values, out=out)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        plan.apply(values, out=out)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))
    flop = encode_flop((N, N, N), (n, n, n))
    tf = flop / (ms * 1e-3) / 1e12
    # bytes: F (FP32) read; axis 0 writes y, reads it back and writes x; the
    # x_1 product reads x and writes Y1; the x_2 product reads Y1, writes P
    nbytes = 4 * N ** 3 + 3 * 8 * n * N * N + 8 * n * N * N + 2 * 8 * n * n * N + 8 * n ** 3
    gbs = nbytes / (ms * 1e-3) / 1e9
    print(json.dumps({
        "metric": "encoded samples/s (fixed-knot least-squares fit)", "value": N ** 3 / (ms * 1e-3),
        "unit": "samples/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64 (f32 samples)",
        "data": "synthetic",
        "config": {"workload": f"{N}^3 FP32 samples of the 64-Gaussian field -> {n}^3 control points, "
                               f"degree {ENC_P}, clamped uniform knots (compression ratio "
                               f"{(N / n) ** 3:.2f}); plan once, timed applies",
                   "plan_ms_host": plan_ms, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gbs / PEAK_HBM_GBS, "traffic": None,
                     "kernel": "one apply: band_fit0_k (axis 0) + gemm_f64_k (axes 1, 2)",
                     "bytes_per_launch": nbytes,
                     "dense_equivalent_tflops": tf,
                     "dense_equivalent_flop": flop},
        "cpu_baseline": cpu}), flush=True)
    return 0


# ------------------------------------------------------------------ isosurface workload
ISO_FRAC = 0.3          # level: 30 % of the control-point range


def flop_per_value(p: int) -> int:
    """Value-only sample: basis values (Horner, p FMAs per function and axis)
    and the sum-factorised contraction (q^3 + q^2 + q FMAs)."""
    q = p + 1
    return 2 * (q ** 3 + q ** 2 + q) + 2 * 3 * q * p


def _iso_cpu_baseline(spec, cam, params, iso, rgb):
    """The FP64 oracle on the central 64 x 64 pixels of the frame."""
    from oracle import render as orr
    c0 = FRAME // 2 - 32
    jj, ii = np.meshgrid(np.arange(c0, c0 + 64), np.arange(c0, c0 + 64), indexing="ij")
    pix = np.stack([jj.reshape(-1), ii.reshape(-1)], axis=1)
    t0 = time.perf_counter()
    r = orr.render_iso(orr.model_field(spec), spec.lo, spec.hi, cam, params, FRAME, FRAME, iso, rgb,
                       pixels=pix)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": len(pix) / dt / FRAME ** 2, "unit": "frames/s", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 NumPy oracle, central 64x64 pixels of the frame ({int((r['hit'] >= 0).sum())} "
                      f"hits) in {dt:.1f} s, scaled to the 1024^2 frame", "cpu_model": _cpu_model()}


def run_iso(args):
    """First-hit isosurface of the 128^3 model's 1024^2 perspective frame at
    30 % of the value range: one launch of iso_k per step."""
    steps = 20 if args.steps is None else args.steps
    spec = synth.model_c2()
    p = spec.blocks[0].degree[0]
    cam = synth.perspective_camera(FRAME, FRAME)
    params = synth.render_params(spec)
    lo, hi = spec.ctrl_min_max()
    iso = float(np.float32(lo + ISO_FRAC * (hi - lo)))
    rgb = (0.9, 0.7, 0.4)
    cpu = None if args.no_cpu_baseline else _iso_cpu_baseline(spec, cam, params, iso, rgb)
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    model = mfa.Model(spec, args.storage)
    rgba = torch.empty((FRAME, FRAME, 4), dtype=torch.float32, device=dev)
    depth = torch.empty((FRAME, FRAME), dtype=torch.float64, device=dev)
    _, _, ns, ne = mfa.render_iso(model, cam, params, FRAME, FRAME, iso, rgb, debug=True, device=dev)
    torch.cuda.synchronize()
    hits = int((ns[..., 1] >= 0).sum().item())
    n_eval = int(ne.sum().item())
    examined = int(torch.where(ns[..., 1] >= 0, ns[..., 1] + 1, ns[..., 0]).sum().item())
    del ns, ne
    for _ in range(args.warmup):
        mfa.render_iso(model, cam, params, FRAME, FRAME, iso, rgb, out=rgba, depth=depth, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        mfa.render_iso(model, cam, params, FRAME, FRAME, iso, rgb, out=rgba, depth=depth, device=dev)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t0) / steps
    ms = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))
    # value-only work for every evaluation but the one full value + gradient
    # evaluation and shading (30 flop) per hit
    flop = (n_eval - hits) * flop_per_value(p) + hits * (flop_per_sample(p) + 30)
    tf = flop / (ms * 1e-3) / 1e12
    print(json.dumps({
        "metric": "isosurface frames/s (1024^2, first hit)", "value": 1e3 / wall_ms,
        "unit": "frames/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": wall_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"f32 ({args.storage} storage)", "data": "synthetic",
        "config": {"workload": f"128^3 model (64-Gaussian field, p = {p}), 1024^2 perspective frame, "
                               f"isosurface at {ISO_FRAC:.0%} of the value range",
                   "kernel_ms": ms, "hits": hits, "samples_examined": examined,
                   "values_evaluated": n_eval, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": tf / PEAK_FP32_TFLOPS, "traffic": None,
                     "peak_unpacked_fp32": PEAK_FP32_ISSUABLE_TFLOPS,
                     "frac_unpacked_fp32": tf / PEAK_FP32_ISSUABLE_TFLOPS,
                     "kernel": "iso_k", "flop_per_launch": flop},
        "cpu_baseline": cpu}), flush=True)
    return 0


# ------------------------------------------------------------------ quality study workload
QUALITY_N, QUALITY_FRAME = 256, 768


def _psnr8(img, ref):
    """PSNR (dB) of two premultiplied RGBA frames over black, as 8-bit RGB
    levels: 10 log10(255^2 / MSE)."""
    a = np.rint(np.clip(img[..., :3], 0.0, 1.0) * 255.0)
    b = np.rint(np.clip(ref[..., :3], 0.0, 1.0) * 255.0)
    m = float(np.mean((a - b) ** 2))
    return (float("inf") if m == 0.0 else 10.0 * np.log10(255.0 ** 2 / m)), m


def run_quality(args):
    """Rendering quality and speed on the Marschner-Lobb function (the
    paper's Sec. V-A1 and Table II setting): 256^3 FP32 samples on [0, 7]^3;
    768^2 perspective frames of the analytic field (ground truth), of the
    samples through the trilinear, Catmull-Rom and cubic B-spline filters,
    and of MFA models (degree 2) fitted to the samples with 256^3 and 128^3
    control points; PSNR of each against the ground truth, ms per frame."""
    steps = 5 if args.steps is None else args.steps
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    N, S = QUALITY_N, QUALITY_FRAME
    lo, hi = (0.0, 0.0, 0.0), (7.0, 7.0, 7.0)
    vol = torch.as_tensor(synth.marschner_lobb_samples(N)).to(dev)
    cam = synth.perspective_camera(S, S, az_deg=30.0, el_deg=35.0, dist=15.0, centre=(3.5, 3.5, 3.5))
    params = dict(tf=synth.tf_table_A(), vmin=np.float32(0.0), vmax=np.float32(1.0),
                  step=0.5 * 7.0 / (N - 1), max_samples=2048, ert_alpha=np.float32(0.99),
                  ka=np.float32(0.3), kd=np.float32(0.6), ks=np.float32(0.3),
                  g0=np.float32(0.01), shininess=16)
    tf = torch.as_tensor(params["tf"], device=dev)
    out = torch.empty((S, S, 4), dtype=torch.float32, device=dev)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for k in range(steps):
            fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))

    def vol_fn(kind, v):
        return lambda: mfa.render_volume(v, kind, lo, hi, cam, params, S, S, dims=(N, N, N),
                                         tf_dev=tf, out=out, device=dev)

    results = {}
    ms = timed(vol_fn("marschner_lobb", None))
    gt = out.cpu().numpy().copy()
    results["ground truth (analytic, FP32)"] = dict(ms=ms)
    for kind in ("trilinear", "catmull_rom", "cubic_bspline"):
        ms = timed(vol_fn(kind, vol))
        ps, m = _psnr8(out.cpu().numpy(), gt)
        results[f"{kind} on {N}^3 samples"] = dict(ms=ms, psnr=ps, mse=m, bytes=4 * N ** 3)
    axis = np.arange(N, dtype=np.float64) / (N - 1)
    mfa_rows = {}
    for n in (N, N // 2):
        P = mfa.encode_grid(vol, [axis] * 3, (2, 2, 2), (n, n, n)).cpu().numpy()
        spec = synth.single_block_model(P, [2, 2, 2], None, lo=lo, hi=hi, voxel=7.0 / (N - 1))
        del P
        with mfa.Model(spec, "f32") as M:
            _, ns, ne = mfa.render_frame(M, cam, params, S, S, tf_dev=tf, nsamp=True, neval=True,
                                         device=dev)
            s_eval = int(ne.sum().item())
            ms = timed(lambda: mfa.render_frame(M, cam, params, S, S, tf_dev=tf, out=out, device=dev))
            ps, m = _psnr8(out.cpu().numpy(), gt)
            info = M.info()
        key = f"MFA p=2, {n}^3 control points (compression {(N / n) ** 3:.0f})"
        results[key] = dict(ms=ms, psnr=ps, mse=m, bytes=info["device_bytes"], evaluated=s_eval)
        mfa_rows[n] = key
        del spec
    comp = results[mfa_rows[N // 2]]
    fl = (flop_per_sample(2) + 54) * comp["evaluated"]
    tfl = fl / (comp["ms"] * 1e-3) / 1e12
    print(json.dumps({
        "metric": "PSNR (dB) of a 768^2 Marschner-Lobb frame against the analytic field",
        "value": comp["psnr"], "unit": "dB", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": comp["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Marschner-Lobb (f_M = 6, alpha = 0.25) on [0, 7]^3 sampled at {N}^3 "
                               f"FP32, {S}^2 perspective frames; value: MFA with {N // 2}^3 control "
                               f"points", "methods": results, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": tfl, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": tfl / PEAK_FP32_TFLOPS, "traffic": None,
                     "peak_unpacked_fp32": PEAK_FP32_ISSUABLE_TFLOPS,
                     "frac_unpacked_fp32": tfl / PEAK_FP32_ISSUABLE_TFLOPS,
                     "kernel": "render_k (MFA model, 128^3 control points)", "flop_per_launch": fl},
        "cpu_baseline": None}), flush=True)
    return 0


# ------------------------------------------------------------------ object-space split workload
def run_composite(args):
    """The object-space split of the 8x8x8-block model's 2048^2 frame: eight
    partial renders of 4x4x4-block octants (each one GPU's share of an
    8-GPU split) and the depth-ordered "over" of the eight partial images,
    against the single full frame."""
    steps = 5 if args.steps is None else args.steps
    spec = synth.model_c4()
    cam = synth.perspective_camera(MB_FRAME, MB_FRAME)
    params = synth.render_params(spec, max_samples=2048)
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    model = mfa.Model(spec, args.storage)
    tf = torch.as_tensor(params["tf"], device=dev)
    S = MB_FRAME
    half = [g // 2 for g in spec.grid]
    boxes = []
    for o in range(8):
        lo = [half[a] * ((o >> (2 - a)) & 1) for a in range(3)]
        boxes.append((lo, [lo[a] + half[a] for a in range(3)]))
    imgs = [torch.empty((S, S, 4), dtype=torch.float32, device=dev) for _ in boxes]
    keys = [torch.empty((S, S), dtype=torch.float64, device=dev) for _ in boxes]
    comp = torch.empty((S, S, 4), dtype=torch.float32, device=dev)
    full = torch.empty((S, S, 4), dtype=torch.float32, device=dev)

    def step(ev=None):
        for g, (lo, hi) in enumerate(boxes):
            mfa.render_partial(model, cam, params, S, S, lo, hi, tf_dev=tf, out=imgs[g], key=keys[g],
                               device=dev)
            if ev:
                ev[g + 1].record(stream)
        mfa.composite_over(imgs, keys, out=comp)
        if ev:
            ev[9].record(stream)
        mfa.render_frame(model, cam, params, S, S, tf_dev=tf, out=full, device=dev)
        if ev:
            ev[10].record(stream)

    for _ in range(args.warmup):
        step()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(11)] for _ in range(steps)]
    torch.cuda.synchronize()
    for k in range(steps):
        events[k][0].record(stream)
        step(events[k])
    torch.cuda.synchronize()
    el = lambda i: float(np.mean([events[k][i].elapsed_time(events[k][i + 1]) for k in range(steps)]))
    part_ms = [el(g) for g in range(8)]
    comp_ms, full_ms = el(8), el(9)
    npix = S * S
    comp_bytes = npix * (8 * (16 + 8) + 16)
    gbs = comp_bytes / (comp_ms * 1e-3) / 1e9
    diff = float((comp - full).abs().max().item())
    print(json.dumps({
        "metric": "object-space split: ms per partial frame (one GPU's share) and composite GB/s",
        "value": max(part_ms), "unit": "ms (slowest octant partial render)", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": sum(part_ms) + comp_ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "8x8x8-block model, 2048^2 perspective frame split into 8 octants of "
                               "4x4x4 blocks: 8 partial renders + depth-ordered over of 8 images",
                   "parallelism": "single GPU (the 8 shares run one after another)"},
        "partial_ms": part_ms, "full_frame_ms": full_ms, "composite_ms": comp_ms,
        "composite_vs_full_max_abs": diff,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gbs / PEAK_HBM_GBS, "traffic": None, "kernel": "composite_k",
                     "bytes_per_launch": comp_bytes}}), flush=True)
    model.close()
    return 0


# ------------------------------------------------------------------ serving workload
def _serving_trace(n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        if rng.random() < 0.5:
            side = int(rng.choice([256, 512, 1024, 2048]))
            reqs.append(("render", int(rng.integers(0, 3)), side,
                         float(rng.uniform(0, 360)), float(rng.uniform(-60, 60))))
        else:
            reqs.append(("points", int(rng.integers(0, 3)), int(10 ** rng.uniform(3, 7)), 0.0, 0.0))
    return reqs


def _serve_run(mfa, torch, dev, specs, storages, trace, rate, pools, xyz, tfs, params, batch_items):
    """Submits the trace open-loop (exponential gaps at `rate`; rate 0 = all
    at once) and returns per-request (latency, kind, size) and the wall time."""
    models = [mfa.Model(sp, st) for sp, st in zip(specs, storages)]
    S = mfa.Server(hbm_budget_bytes=200 * 10 ** 9, queue_cap=16384, max_batch_items=batch_items)
    ids = [S.add_model(M) for M in models]
    rng = np.random.default_rng(99)
    gaps = rng.exponential(1.0 / rate, size=len(trace)) if rate > 0 else np.zeros(len(trace))
    sched = np.cumsum(gaps)
    slot_ticket = {}
    tickets = []
    t0 = time.perf_counter()
    for k, (kind, mid, size, az, el) in enumerate(trace):
        delay = t0 + sched[k] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        key = (kind, size if kind == "render" else 0, k % len(pools[kind, size if kind == "render" else 0]))
        if key in slot_ticket:                          # buffer reuse waits for its last user
            S.wait(slot_ticket[key])
        buf = pools[key[0], key[1]][key[2]]
        lag = time.perf_counter() - (t0 + sched[k])
        if kind == "render":
            cam = synth.perspective_camera(size, size, az_deg=az, el_deg=el)
            t = S.submit_render(ids[mid], cam, params[mid], size, size, buf, tf_dev=tfs[mid])
        else:
            t = S.submit_points(ids[mid], xyz, buf, n=size)     # first 3*size floats of xyz
        slot_ticket[key] = t
        tickets.append((t, lag, kind, size))
    out = []
    for t, lag, kind, size in tickets:
        st = S.wait(t)
        out.append((st["t_done"] - st["t_submit"] + lag, kind, size))
    wall = time.perf_counter() - t0
    S.close()
    for M in models:
        M.close()
    return out, wall


def run_serving(args):
    """Open-loop Poisson trace over three resident models: the 16^3 model in
    FP32, the same in BF16 and the 48^3 least-squares model in BF16 (and a
    plain run with all three in FP32).  Half the requests are renders of
    256^2..2048^2 from random orbit cameras, half are point batches of
    10^3..10^7 points."""
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    c1 = synth.model_c1()
    c48 = synth.model_c3_fit48()
    specs = [c1, c1, c48]
    params = [synth.render_params(sp) for sp in specs]
    tfs = [torch.as_tensor(p["tf"], device=dev) for p in params]
    nmax = 10 ** 7
    xyz = torch.as_tensor(synth.random_points(nmax, seed=5), device=dev)
    nslot = 24
    pools = {("render", s): [torch.empty((s, s, 4), device=dev) for _ in range(nslot)]
             for s in (256, 512, 1024, 2048)}
    pools["points", 0] = [torch.empty((nmax, 4), device=dev) for _ in range(nslot)]
    warm = max(50, args.requests // 20)
    trace = _serving_trace(warm + args.requests, seed=5)
    # capacity: the whole trace at once (closed burst)
    burst = trace[:min(400, len(trace))]
    _, wall = _serve_run(mfa, torch, dev, specs, ["f32", "bf16", "bf16"], burst, 0.0, pools, xyz,
                         tfs, params, args.batch_items)
    capacity = len(burst) / wall
    rate = args.load * capacity
    res = {}
    for label, storages in (("bf16_mix", ["f32", "bf16", "bf16"]), ("fp32", ["f32", "f32", "f32"])):
        lat, wall = _serve_run(mfa, torch, dev, specs, storages, trace, rate, pools, xyz, tfs, params,
                               args.batch_items)
        lat = lat[warm:]
        ms = np.array([x[0] for x in lat]) * 1e3
        kinds = np.array([x[1] for x in lat])
        res[label] = {"p50_ms": float(np.percentile(ms, 50)), "p99_ms": float(np.percentile(ms, 99)),
                      "p50_render_ms": float(np.percentile(ms[kinds == "render"], 50)),
                      "p99_render_ms": float(np.percentile(ms[kinds == "render"], 99)),
                      "p50_points_ms": float(np.percentile(ms[kinds == "points"], 50)),
                      "p99_points_ms": float(np.percentile(ms[kinds == "points"], 99)),
                      "throughput_rps": len(trace) / wall}
    print(json.dumps({
        "metric": METRIC, "value": res["bf16_mix"]["p99_ms"], "unit": "ms (p99 latency)",
        "n_gpus": 1, "steps": args.requests, "warmup": warm, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (bf16 storage for 2 of 3 models)",
        "data": "synthetic",
        "config": {"workload": ("serving: 16^3 FP32, 16^3 BF16 and 48^3 BF16 models resident, "
                                "open-loop Poisson arrivals, 50 % renders 256^2..2048^2, 50 % point "
                                "batches 1e3..1e7, 200 GB budget"),
                   "capacity_rps": capacity, "offered_rps": rate, "load": args.load,
                   "batch_items": args.batch_items, "measured_requests": args.requests,
                   "parallelism": "single GPU"},
        "serving": res,
        "p99_bf16_over_fp32": res["bf16_mix"]["p99_ms"] / res["fp32"]["p99_ms"]}), flush=True)
    return 0



# ------------------------------------------------------------------ storage-form comparison
def _image_errors(img, ref):
    """RMSE over RGBA and 8-bit PSNR over RGB of sampled pixels (m, 4)."""
    rmse = float(np.sqrt(np.mean((img.astype(np.float64) - ref) ** 2)))
    return rmse, _psnr8(img, ref)[0]


def _storage_case(args, name, spec, field, step_fn_factory, frame, params, n_pix, seed):
    """Kernel times of one step per storage form, and the image error of
    the frame on n_pix sampled pixels against the FP64 oracle (FP64 control
    points) and against the analytic field rendered by the same oracle
    renderer (the ground truth of the paper's image-error comparison)."""
    import torch
    import paper_2312_15073_amd as mfa
    from oracle import render as orr
    dev = torch.device("cuda:0")
    steps = 10 if args.steps is None else args.steps
    cam = synth.perspective_camera(frame, frame)
    rng = np.random.default_rng(seed)
    pix = np.stack([rng.integers(0, frame, n_pix), rng.integers(0, frame, n_pix)], axis=1)
    flat = pix[:, 0] * frame + pix[:, 1]
    t0 = time.perf_counter()
    ref = orr.render(orr.model_field(spec), spec.lo, spec.hi, cam, params, frame, frame,
                     pixels=pix)["rgba"]
    gt = orr.render(lambda x: field.value_grad(x), spec.lo, spec.hi, cam, params, frame, frame,
                    pixels=pix)["rgba"]
    t_oracle = time.perf_counter() - t0
    rows = {}
    for storage in ("f32", "bf16", "f16"):
        model = mfa.Model(spec, storage)
        names, step = step_fn_factory(model, cam)
        for _ in range(args.warmup):
            step(None)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)]
               for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step(evs[k])
        torch.cuda.synchronize()
        ms_step = 1e3 * (time.perf_counter() - t0) / steps
        kms = {n: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(steps)]))
               for i, n in enumerate(names)}
        tf = torch.as_tensor(params["tf"], device=dev)
        img = mfa.render_frame(model, cam, params, frame, frame, tf_dev=tf, device=dev)
        img = img.cpu().numpy().reshape(-1, 4)[flat]
        e_or, p_or = _image_errors(img, ref)
        e_gt, p_gt = _image_errors(img, gt)
        rows[storage] = dict(ms_step=ms_step, kernels_ms=kms, ctrl_bytes=model.info()["ctrl_bytes"],
                             image_rmse_vs_fp64_oracle=e_or, image_psnr8_vs_fp64_oracle=p_or,
                             image_rmse_vs_ground_truth=e_gt, image_psnr8_vs_ground_truth=p_gt)
        model.close()
    f32 = rows["f32"]
    for storage, r in rows.items():
        r["speedup_vs_f32_step"] = f32["ms_step"] / r["ms_step"]
        r["speedup_vs_f32_kernels"] = {k: f32["kernels_ms"][k] / v for k, v in r["kernels_ms"].items()}
        r["equal_image_error_to_f32"] = bool(
            r["image_rmse_vs_ground_truth"] <= 1.05 * f32["image_rmse_vs_ground_truth"]
            or abs(r["image_psnr8_vs_ground_truth"] - f32["image_psnr8_vs_ground_truth"]) <= 0.1)
    return {"model": name, "sampled_pixels": n_pix, "oracle_seconds": t_oracle, "forms": rows}


def run_storage(args):
    """FP32 against BF16 and FP16 control-point storage on the 128^3 step
    (512^3 grid + 1e7 sorted points + 1024^2 frame) and the 8x8x8-block step
    (1e8 sorted points + 2048^2 frame): per-kernel times and the speedup of
    each form at the image error it reaches (Table II's comparison against
    the analytic field)."""
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    out = []
    if args.storage_model in ("both", "single128"):
        spec = synth.model_c2()
        params = synth.render_params(spec)
        xyz = torch.as_tensor(synth.random_points(N_POINTS, seed=12), device=dev)
        axes = [torch.as_tensor(synth.grid_axis(GRID_N), device=dev) for _ in range(3)]
        grid_out = torch.empty((GRID_N, GRID_N, GRID_N, 4), dtype=torch.float32, device=dev)
        pts_out = torch.empty((N_POINTS, 4), dtype=torch.float32, device=dev)
        rgba = torch.empty((FRAME, FRAME, 4), dtype=torch.float32, device=dev)
        tf = torch.as_tensor(params["tf"], device=dev)

        def factory(model, cam):
            def step(ev):
                if ev is not None:
                    ev[0].record(stream)
                mfa.decode_grid(model, axes, out=grid_out)
                if ev is not None:
                    ev[1].record(stream)
                mfa.decode_points(model, xyz, out=pts_out, sorted_order=True)
                if ev is not None:
                    ev[2].record(stream)
                mfa.render_frame(model, cam, params, FRAME, FRAME, tf_dev=tf, out=rgba, device=dev)
                if ev is not None:
                    ev[3].record(stream)
            return ["decode_grid", "decode_points", "render"], step

        out.append(_storage_case(args, "single block, 128^3 control points, degree 3", spec,
                                 synth.field_c2(), factory, FRAME, params, 1024, 31))
        del grid_out, pts_out, xyz
        torch.cuda.empty_cache()
    if args.storage_model in ("both", "multiblock"):
        spec = synth.model_c4()
        params = synth.render_params(spec, max_samples=2048)
        xyz = torch.as_tensor(synth.random_points(MB_POINTS, seed=14), device=dev)
        pts_out = torch.empty((MB_POINTS, 4), dtype=torch.float32, device=dev)
        rgba = torch.empty((MB_FRAME, MB_FRAME, 4), dtype=torch.float32, device=dev)
        tf = torch.as_tensor(params["tf"], device=dev)

        def factory(model, cam):
            def step(ev):
                if ev is not None:
                    ev[0].record(stream)
                mfa.decode_points(model, xyz, out=pts_out, sorted_order=True)
                if ev is not None:
                    ev[1].record(stream)
                mfa.render_frame(model, cam, params, MB_FRAME, MB_FRAME, tf_dev=tf, out=rgba, device=dev)
                if ev is not None:
                    ev[2].record(stream)
            return ["decode_points", "render"], step

        out.append(_storage_case(args, "8x8x8 blocks, 56.8M control points, degree 3", spec,
                                 synth.turbulence_field(512, 104), factory, MB_FRAME, params, 384, 32))
    c = out[0]
    bf = c["forms"]["bf16"]
    print(json.dumps({
        "metric": "speedup of BF16 control-point storage over FP32 (step time) at the image error it reaches",
        "value": bf["speedup_vs_f32_step"], "unit": "x", "n_gpus": 1,
        "steps": 10 if args.steps is None else args.steps, "warmup": args.warmup,
        "ms_per_step": bf["ms_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f32 / bf16 / f16 storage)", "data": "synthetic",
        "config": {"workload": "storage forms on the 128^3 step and the 8x8x8-block step",
                   "cases": out, "parallelism": "single GPU"},
        "cpu_baseline": None}), flush=True)
    return 0


# ------------------------------------------------------------------ value-only queries
def run_values(args):
    """Value-only against value+gradient queries (the paper's Fig. 8a and
    8b) on the 128^3 model: the 512^3 grid and 1e7 random points (sorted)."""
    steps = 10 if args.steps is None else args.steps
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    spec = synth.model_c2()
    model = mfa.Model(spec, args.storage)
    axes = [torch.as_tensor(synth.grid_axis(GRID_N), device=dev) for _ in range(3)]
    xyz = torch.as_tensor(synth.random_points(N_POINTS, seed=12), device=dev)
    g4 = torch.empty((GRID_N, GRID_N, GRID_N, 4), dtype=torch.float32, device=dev)
    g1 = torch.empty((GRID_N, GRID_N, GRID_N), dtype=torch.float32, device=dev)
    p4 = torch.empty((N_POINTS, 4), dtype=torch.float32, device=dev)
    p1 = torch.empty((N_POINTS,), dtype=torch.float32, device=dev)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for k in range(steps):
            fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))

    rows = {
        "grid value+gradient": (timed(lambda: mfa.decode_grid(model, axes, out=g4)), GRID_N ** 3, 16),
        "grid value": (timed(lambda: mfa.decode_grid(model, axes, out=g1, value_only=True)), GRID_N ** 3, 4),
        "points value+gradient (sorted)": (timed(lambda: mfa.decode_points(model, xyz, out=p4, sorted_order=True)),
                                           N_POINTS, 28),
        "points value (sorted)": (timed(lambda: mfa.decode_points(model, xyz, out=p1, sorted_order=True,
                                                                  value_only=True)), N_POINTS, 16),
        "points value+gradient (input order)": (timed(lambda: mfa.decode_points(model, xyz, out=p4)),
                                                N_POINTS, 28),
        "points value (input order)": (timed(lambda: mfa.decode_points(model, xyz, out=p1, value_only=True)),
                                       N_POINTS, 16),
    }
    res = {k: dict(ms=ms, samples_per_s=n / (ms * 1e-3), hbm_gbs=(n * b + model.info()["ctrl_bytes"]) / (ms * 1e6),
                   bytes_per_unit=b) for k, (ms, n, b) in rows.items()}
    tot_ms = res["grid value"]["ms"] + res["points value (sorted)"]["ms"]
    print(json.dumps({
        "metric": "value-only queries/s (grid + sorted points)",
        "value": (GRID_N ** 3 + N_POINTS) / (tot_ms * 1e-3), "unit": "samples/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": tot_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"f32 ({args.storage} storage)", "data": "synthetic",
        "config": {"workload": f"128^3 model, degree 3: {GRID_N}^3 grid and {N_POINTS} random points, "
                               "value only against value + gradient", "queries": res,
                   "parallelism": "single GPU"},
        "cpu_baseline": None}), flush=True)
    model.close()
    return 0


# ------------------------------------------------------------------ compression-ratio sweep
def run_cr_sweep(args):
    """Marschner-Lobb 256^3 samples (Sec. V-A1 function on [0, 7]^3)
    encoded by the fixed-knot least-squares fit (degree 2) at control-point
    counts n^3 giving compression ratios (256/n)^3 of about 20, 69, 134 and
    212 (the ratios of Fig. 5), plus 128^3 (8) and 256^3 (1) for reference:
    encode time, the 768^2 frame time and its PSNR against the analytic
    field."""
    steps = 5 if args.steps is None else args.steps
    import torch
    import paper_2312_15073_amd as mfa
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    N, S = QUALITY_N, QUALITY_FRAME
    lo, hi = (0.0, 0.0, 0.0), (7.0, 7.0, 7.0)
    vol = torch.as_tensor(synth.marschner_lobb_samples(N)).to(dev)
    cam = synth.perspective_camera(S, S, az_deg=30.0, el_deg=35.0, dist=15.0, centre=(3.5, 3.5, 3.5))
    params = dict(tf=synth.tf_table_A(), vmin=np.float32(0.0), vmax=np.float32(1.0),
                  step=0.5 * 7.0 / (N - 1), max_samples=2048, ert_alpha=np.float32(0.99),
                  ka=np.float32(0.3), kd=np.float32(0.6), ks=np.float32(0.3),
                  g0=np.float32(0.01), shininess=16)
    tf = torch.as_tensor(params["tf"], device=dev)
    out = torch.empty((S, S, 4), dtype=torch.float32, device=dev)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for k in range(steps):
            fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))

    mfa.render_volume(None, "marschner_lobb", lo, hi, cam, params, S, S, dims=(N, N, N), tf_dev=tf,
                      out=out, device=dev)
    gt = out.cpu().numpy().copy()
    axis = np.arange(N, dtype=np.float64) / (N - 1)
    rows = []
    for n in (256, 128, 94, 62, 50, 43):
        plan = mfa.EncodePlan((N, N, N), [axis] * 3, (2, 2, 2), (n, n, n))
        P = plan.apply(vol)
        ms_enc = timed(lambda: plan.apply(vol, out=P))
        Ph = P.cpu().numpy()
        del plan
        fl = encode_flop((N, N, N), (n, n, n))
        spec = synth.single_block_model(Ph, [2, 2, 2], None, lo=lo, hi=hi, voxel=7.0 / (N - 1))
        with mfa.Model(spec, "f32") as M:
            _, ns, ne = mfa.render_frame(M, cam, params, S, S, tf_dev=tf, nsamp=True, neval=True,
                                         device=dev)
            s_eval = int(ne.sum().item())
            ms = timed(lambda: mfa.render_frame(M, cam, params, S, S, tf_dev=tf, out=out, device=dev))
            ps, m = _psnr8(out.cpu().numpy(), gt)
        rows.append(dict(n_ctrl=n, compression_ratio=(N / n) ** 3, encode_ms=ms_enc,
                         encode_tflops_dense=fl / (ms_enc * 1e-3) / 1e12,
                         encode_hbm_gbs=_encode_bytes((N, N, N), (n, n, n)) / (ms_enc * 1e6),
                         ms_per_frame=ms, psnr8=ps, mse8=m, evaluated_samples=s_eval,
                         render_tflops=s_eval * (flop_per_sample(2) + 54) / (ms * 1e-3) / 1e12))
        del P, spec
    r20 = next(r for r in rows if r["n_ctrl"] == 94)
    print(json.dumps({
        "metric": "PSNR (dB) of a 768^2 Marschner-Lobb frame at compression ratio 20",
        "value": r20["psnr8"], "unit": "dB", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": r20["ms_per_frame"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (FP64 encode)", "data": "synthetic",
        "config": {"workload": f"Marschner-Lobb {N}^3 FP32 samples on [0, 7]^3, degree 2 fits at "
                               f"n^3 control points, {S}^2 perspective frames", "sweep": rows,
                   "parallelism": "single GPU"},
        "cpu_baseline": None}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
