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
over the step, counting the grid points, the random points and every sample
the frame composites.
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args(argv)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU path is a design, not part of this build", file=sys.stderr)
        return 2

    spec = synth.model_c2()
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
    samples_step = n_grid + N_POINTS + s_frame

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
    model_bytes = info["device_bytes"]
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
                "unit": dk["unit"], "frac": dk["frac"], "traffic": None, "kernel": dom}
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
        "config": {"workload": (f"single block, {spec.blocks[0].ctrl.shape[0]}^3 control points, "
                                f"degree {p}, {args.storage} storage; decode {GRID_N}^3 grid + "
                                f"{N_POINTS} random points + {FRAME}x{FRAME} perspective frame "
                                f"(max 1024 samples/ray)"),
                   "samples_per_step": samples_step, "frame_samples": s_frame,
                   "frame_samples_evaluated": s_eval,
                   "parallelism": "single GPU"},
        "ms_per_frame": kern_ms["render"],
        "kernels": kernels,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    model.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
