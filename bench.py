#!/usr/bin/env python3
"""Benchmark of the lens transport hot path on one MI355X.

Workload: the 11-surface double-Gauss-style lens with 4,194,304 sensor-side
rays (sensor uniform on 36 x 24 mm, directions uniform toward the rear
element, wavelength uniform in 400..700 nm), inputs resident in HBM.  One
step = one pass of the hot path over the batch: the brute-force trace of the
transmit path (lt_trace) and, when a map is available, its fused network
evaluation (lt_map_eval).

Prints one JSON line (see the keys below).  Kernel times are taken with HIP
events on the stream the kernels are launched on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_RAYS = 4194304
MI355X_FP32_VECTOR_TFLOPS = 157.3
MI355X_BF16_MFMA_TFLOPS = 2500.0
MI355X_FP8_MFMA_TFLOPS = 5000.0
MI355X_HBM_GBS = 8000.0
MAP_WIDTH, MAP_DEPTH = 128, 5


def map_flops_per_ray(width=MAP_WIDTH, depth=MAP_DEPTH, heads=1):
    """Algorithmic flops of one network evaluation (2 per multiply-add):
    6 -> width, (depth - 1) x width -> width, width -> 6 * heads."""
    return 2 * (6 * width + (depth - 1) * width * width + width * 6 * heads)


def trace_flops_per_ray(lens, path=(0, 0, 0)):
    """Algorithmic FP32 operations of one ray along a path, counted on the
    plain single-rounding algorithm (FMA = 2, add/mul/compare = 1, sqrt/div =
    1): 20 for set-up, 78 per refraction, 56 per reflection, 28 per stop
    crossing, 10 for the exit plane."""
    surfs = lens.surfaces
    n_stop = sum(s.is_stop for s in surfs)
    nr = len(surfs) - n_stop
    if path[0] == 0:
        n_t, n_r, n_s = nr, 0, n_stop
    else:
        j, i = path[1], path[2]
        n_t, n_r = nr + 2 * (i - j) - 2, 2
        n_s = n_stop  # ghost paths cross the stop at least once; counted once
    return 20 + 78 * n_t + 56 * n_r + 28 * n_s + 10


def cpu_baseline_map(params, rays_np, budget_s=10.0):
    """Time the FP64 reference network (numpy) on a bounded sample."""
    from oracle import mlp
    threads = os.cpu_count() or 1
    n = 16384
    while True:
        sample = {k: v[:n] for k, v in rays_np.items()}
        t0 = time.perf_counter()
        o, _ = mlp.forward(params, mlp.features(sample, params))
        mlp.decode(o, params)
        dt = time.perf_counter() - t0
        if dt > budget_s / 4 or n * 4 > rays_np["x"].shape[0]:
            break
        n *= 4
    return {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} rays, FP64 numpy forward of the 5 x 128 tanh map "
                      f"(BLAS threads = host cores)"}


def cpu_baseline(lens, rays_np, budget_s=10.0):
    """Time the FP64 oracle on the host cores on a bounded sample."""
    import oracle
    n_all = rays_np["x"].shape[0]
    threads = os.cpu_count() or 1
    probe = {k: v[:65536] for k, v in rays_np.items()}
    t0 = time.perf_counter()
    oracle.trace(lens, probe, nthreads=threads)
    dt = time.perf_counter() - t0
    n = int(min(n_all, max(65536, 65536 * budget_s / max(dt, 1e-6))))
    sample = {k: v[:n] for k, v in rays_np.items()}
    t0 = time.perf_counter()
    oracle.trace(lens, sample, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of the {n_all} rays, transmit path, FP64 C oracle, OpenMP"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rays", type=int, default=N_RAYS)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every box in this setup has one MI355X; "
              "multi-GPU sharding is described in DESIGN.md, not run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2605_04017_amd as lt
    import synth

    dev = torch.device("cuda:0")
    lens = synth.config_lens(2)
    rays_np = synth.config_rays(2, args.rays)
    n = args.rays
    rays = {k: torch.from_numpy(v).to(dev) for k, v in rays_np.items()}
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    out = lt.empty_exit(n, dev)
    out_fast = lt.empty_exit(n, dev)
    stream = torch.cuda.current_stream()

    # map of the workload's architecture: 6-D input, 5 x 128 tanh, one head
    from oracle import mlp
    desc = mlp.MapDesc(MAP_WIDTH, MAP_DEPTH, 1, mlp.ACT_TANH)
    params = mlp.init_params(desc, 7)
    x = np.stack([rays_np[k][:65536].astype(np.float64) for k in synth.RAY_FIELDS], 1)
    params.in_shift, params.in_scale = x.mean(0), 1.0 / x.std(0)
    m = lt.lt_map_create(MAP_WIDTH, MAP_DEPTH, 1, lt.LT_ACT_TANH)
    lt.lt_map_set_params(m, torch.from_numpy(params.flat().astype(np.float32)).to(dev))
    lt.lt_map_set_norm(m, params.in_shift, params.in_scale, params.out_shift.reshape(-1),
                       params.out_scale.reshape(-1))
    mout = lt.empty_map_out(1, n, dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        lt.lt_trace(h, (0, 0, 0), rays, out, n, stream)
        if ev is not None:
            ev[1].record(stream)
        lt.lt_map_eval(m, lt.LT_BF16, rays, mout, n, stream)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trace_ms = [e[0].elapsed_time(e[1]) for e in evs]
    map_ms = [e[1].elapsed_time(e[2]) for e in evs]
    t_trace = float(np.mean(trace_ms)) * 1e-3
    t_map = float(np.mean(map_ms)) * 1e-3
    ms_per_step = wall / args.steps * 1e3

    # the plain-FP32 tracer option, timed outside the steps for context
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lt.lt_trace_ex(h, (0, 0, 0), rays, out_fast, n, lt.LT_TRACE_PLAIN_FP32, stream)
    e0.record(stream)
    for _ in range(5):
        lt.lt_trace_ex(h, (0, 0, 0), rays, out_fast, n, lt.LT_TRACE_PLAIN_FP32, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_fast = e0.elapsed_time(e1) / 5 * 1e-3

    map_flops = map_flops_per_ray() * n
    achieved = map_flops / t_map / 1e12
    trace_tf = trace_flops_per_ray(lens) * n / t_trace / 1e12
    res = {
        "metric": "Mrays/s map vs GPU brute-force trace at stated exit-ray error; p99 latency",
        "value": n / t_map / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "double-Gauss-style 11-surface lens + stop, 4,194,304 sensor-side "
                               "rays; step = FP32 brute-force trace + 5 x 128 tanh map (BF16 MFMA)",
                   "rays": n, "map": "6-D input, 5 x 128 tanh, 1 head (mask logit + x, y, dx, dy, "
                                     "throughput)"},
        "map_mrays_s": n / t_map / 1e6,
        "trace_mrays_s": n / t_trace / 1e6,
        "trace_plain_fp32_mrays_s": n / t_fast / 1e6,
        "map_over_trace": t_trace / t_map,
        "map_kernel_ms": t_map * 1e3,
        "trace_kernel_ms": t_trace * 1e3,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MI355X_BF16_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / MI355X_BF16_MFMA_TFLOPS,
                     "traffic": None, "kernel": "map_eval_bf16_kernel<128, tanh>",
                     "flops_per_ray": map_flops_per_ray()},
        "roofline_trace": {"bound": "alu", "achieved": trace_tf, "peak": MI355X_FP32_VECTOR_TFLOPS,
                           "unit": "TFLOP/s", "frac": trace_tf / MI355X_FP32_VECTOR_TFLOPS,
                           "kernel": "trace_kernel<compensated>",
                           "flops_per_ray": trace_flops_per_ray(lens)},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_map(params, rays_np)
        res["cpu_baseline_trace"] = cpu_baseline(lens, rays_np)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
