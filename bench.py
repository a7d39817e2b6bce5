#!/usr/bin/env python3
"""Benchmark of the lens transport hot path on one MI355X.

Workload (the headline): the 11-surface double-Gauss-style lens (seeded
prescription and Cauchy glasses) with 16,777,216 sensor-side rays (sensor
point uniform on the 36 x 24 mm frame, direction uniform toward the rear
element, wavelength uniform in 400..700 nm) and every light path with at
most two reflections: the transmit path and the 55 two-reflection ghosts,
56 paths.  Inputs are resident in HBM.

One step = one pass of the hot path over the batch: the brute-force tracer
on all 56 paths (one compacted launch per path: valid rays only) and the map
(one 5 x 128 tanh trunk with a head per path, canonical input, fitted on
GPU-traced rays of all 56 paths) in FP32 with compacted output (mask bitmap
+ valid rays, Sec. 4.2).  `value` is the map's ray-path evaluations per
second; the tracer's rate, their ratios (against each tracer variant that
meets the tolerance), BF16 and FP8 map rates, the uncompacted rates, the
map's error against the GPU tracer, rooflines, and the other workloads (the
4,194,304-ray transmit-only case, the paper-size pair, training, forward
flare tracing, the sampler, serving with p50/p99 latency) are reported in
the same JSON line.  Kernel times come from HIP events on the stream the
kernels run on.  The oracle runs only in the CPU-baseline leg, which times
it on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from paper_2605_04017_amd import fit as F

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_RAYS = 4194304          # the transmit-only case
N_RAYS_ALL_PATHS = 16777216  # the headline: 56 paths
MI355X_FP32_VECTOR_TFLOPS = 157.3
MI355X_FP64_VECTOR_TFLOPS = 78.6
MI355X_FP32_MFMA_TFLOPS = 157.3
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
        n_s = n_stop
    return 20 + 78 * n_t + 56 * n_r + 28 * n_s + 10


def cpu_baseline_map(flat, norms, rays_np, heads=1, canonical=False, budget_s=10.0):
    """Time the FP64 reference network (numpy) of a fitted map (its flat
    parameters and normalisation) on a bounded sample; the rate counts
    ray-path evaluations (rays x heads)."""
    import numpy as np
    from oracle import mlp
    params = mlp.init_params(mlp.MapDesc(MAP_WIDTH, MAP_DEPTH, heads, mlp.ACT_TANH, canonical=canonical), 0)
    params.set_flat(np.asarray(flat, np.float64))
    params.in_shift, params.in_scale = norms[0], norms[1]
    params.out_shift, params.out_scale = norms[2], norms[3]
    threads = os.cpu_count() or 1
    n = 4096
    while True:
        sample = {k: v[:n] for k, v in rays_np.items()}
        t0 = time.perf_counter()
        o, _ = mlp.forward(params, mlp.features(sample, params))
        mlp.decode(o, params, sample)
        dt = time.perf_counter() - t0
        if dt > budget_s / 4 or n * 4 > rays_np["x"].shape[0]:
            break
        n *= 4
    unit = "Mray-paths/s" if heads > 1 else "Mrays/s"
    return {"value": n * heads / dt / 1e6, "unit": unit, "cores": threads, "kind": "oracle",
            "sample": f"first {n} rays of the workload x {heads} heads, FP64 numpy forward and decode "
                      f"of the 5 x 128 tanh map (BLAS threads = host cores)"}


def cpu_baseline_trace(lens, rays_np, paths=((0, 0, 0),), budget_s=10.0):
    """Time the FP64 oracle tracer on the host cores on a bounded sample of
    rays, each traced along every path in `paths`; the rate counts
    ray-path traces."""
    import oracle
    n_all = rays_np["x"].shape[0]
    threads = os.cpu_count() or 1
    probe = {k: v[:8192] for k, v in rays_np.items()}
    t0 = time.perf_counter()
    for p in paths:
        oracle.trace(lens, probe, p, nthreads=threads)
    dt = time.perf_counter() - t0
    n = int(min(n_all, max(8192, 8192 * budget_s / max(dt, 1e-6))))
    sample = {k: v[:n] for k, v in rays_np.items()}
    t0 = time.perf_counter()
    for p in paths:
        oracle.trace(lens, sample, p, nthreads=threads)
    dt = time.perf_counter() - t0
    what = "transmit path" if len(paths) == 1 else f"all {len(paths)} paths"
    unit = "Mrays/s" if len(paths) == 1 else "Mray-paths/s"
    return {"value": n * len(paths) / dt / 1e6, "unit": unit, "cores": threads, "kind": "oracle",
            "sample": f"first {n} of the {n_all} rays, {what}, FP64 C oracle, OpenMP"}


def time_kernel(fn, stream, reps):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def fit_map(lt, synth, lens, dev, steps, batch=65536, seed=3002, canonical=False):
    """Fit the 5 x 128 tanh map on rays the GPU tracer labels (a fresh
    65,536-ray batch per step drawn from a 4M-ray pool that does not overlap
    the benchmark rays).  canonical: symmetry-reduced input frame (the
    normalisation statistics are then taken in that frame).  Returns (map,
    (flat parameters, normalisation), final loss)."""
    import numpy as np
    import torch
    pool_np = synth.make_rays(lens, 4194304, seed)
    pool = {k: torch.from_numpy(v).to(dev) for k, v in pool_np.items()}
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    ex = lt.lt_trace(h, (0, 0, 0), pool)
    ok = ex["mask"].bool()
    reg = torch.stack([ex[k][ok] for k in ("x", "y", "dx", "dy", "throughput")], 1).double().cpu().numpy()
    norms = F.map_norms(pool_np, [(ok.cpu().numpy(), reg)], canonical)
    m = lt.lt_map_create(MAP_WIDTH, MAP_DEPTH, 1, lt.LT_ACT_TANH, canonical)
    lt.lt_map_set_params(m, torch.from_numpy(F.init_params(MAP_WIDTH, MAP_DEPTH, 1, 5)).to(dev))
    lt.lt_map_set_norm(m, norms[0], norms[1], norms[2].reshape(-1), norms[3].reshape(-1))
    ws = lt.workspace(m, batch)
    n_pool = pool_np["x"].shape[0]
    loss = None
    for k in range(1, steps + 1):
        lo = ((k - 1) * batch) % (n_pool - batch + 1)
        rb = {f: v[lo:lo + batch] for f, v in pool.items()}
        tb = {"valid": ex["mask"][lo:lo + batch].reshape(1, -1)}
        for f in ("x", "y", "dx", "dy", "throughput"):
            tb[f] = ex[f][lo:lo + batch].reshape(1, -1)
        lr = 2e-3 * (0.5 ** (k / max(1, steps / 4)))
        loss = lt.lt_map_train_step(m, rb, tb, {"lr": lr, "step": k, "w_bce": 1.0, "w_l2": 4.0}, ws)
    torch.cuda.synchronize()
    return m, (lt.lt_map_get_params(m).cpu().numpy(), norms), [float(v) for v in loss.cpu()]


def map_error(lt, h, m, dtype, rays_dev, n_sample=65536):
    """Exit-ray error of the map on the first n_sample benchmark rays against
    the FP32 GPU tracer, which matches the FP64 oracle to within 1e-5 mm and
    1e-6 rad (the GPU parity tests; a separate test checks that a fitted
    map's error against both agrees to that bound)."""
    sub = {k: v[:n_sample] for k, v in rays_dev.items()}
    return exit_error(eval_host(lt.lt_map_eval(m, dtype, sub)),
                      {k: v.cpu().numpy() for k, v in lt.lt_trace(h, (0, 0, 0), sub).items()}, n_sample)


def eval_host(out):
    """First head of map outputs as host arrays."""
    return {k: v[0].cpu().numpy() for k, v in out.items()}


def exit_error(g, o, n_sample):
    """Mask agreement and exit-ray errors of map outputs g (one head, host
    arrays) against traced exits o."""
    import numpy as np
    gm, om = g["mask"].astype(bool), o["mask"].astype(bool)
    both = gm & om
    if not both.any():   # a barely fitted classifier may accept nothing
        return {"mask_agreement": float(np.mean(gm == om)), "false_valid": float(np.mean(gm & ~om)),
                "false_invalid": float(np.mean(~gm & om)), "rays": n_sample, "valid_in_both": 0}
    pos = np.hypot(g["x"][both] - o["x"][both], g["y"][both] - o["y"][both])
    u = np.stack([g["dx"][both], g["dy"][both], g["dz"][both]], 1).astype(np.float64)
    v = np.stack([o["dx"][both], o["dy"][both], o["dz"][both]], 1)
    ang = 2 * np.arcsin(np.minimum(1.0, np.linalg.norm(u - v, axis=1) / 2))
    thr = np.abs(g["throughput"][both] - o["throughput"][both])
    return {"mask_agreement": float(np.mean(gm == om)), "false_valid": float(np.mean(gm & ~om)),
            "false_invalid": float(np.mean(~gm & om)),
            "pos_mm_p50": float(np.median(pos)), "pos_mm_p99": float(np.quantile(pos, 0.99)),
            "dir_rad_p50": float(np.median(ang)), "dir_rad_p99": float(np.quantile(ang, 0.99)),
            "throughput_abs_p99": float(np.quantile(thr, 0.99)), "rays": n_sample}


def paper_pair(lt, synth, lens, dev, steps, rays, batch=65536, seed=3003,
               w_cos=200.0):
    """The paper's factorised form at its own size: a classifier of 2 x 32
    tanh (BCE) and a regressor of 5 x 32 tanh (squared error on position and
    throughput, cosine loss on direction), both fitted for `steps` steps on
    GPU-traced rays; evaluation runs the classifier (LT_EVAL_MASK_ONLY) and
    then the regressor under its mask (LT_EVAL_GATED)."""
    import numpy as np
    import torch
    pool_np = synth.make_rays(lens, 4194304, seed)
    pool = {k: torch.from_numpy(v).to(dev) for k, v in pool_np.items()}
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    ex = lt.lt_trace(h, (0, 0, 0), pool)
    ok = ex["mask"].bool()
    reg_t = torch.stack([ex[k][ok] for k in ("x", "y", "dx", "dy", "throughput")], 1).double().cpu().numpy()
    norms = F.map_norms(pool_np, [(ok.cpu().numpy(), reg_t)])
    nets = {}
    for name, depth in (("classifier", 2), ("regressor", 5)):
        m = lt.lt_map_create(32, depth, 1, lt.LT_ACT_TANH)
        lt.lt_map_set_params(m, torch.from_numpy(F.init_params(32, depth, 1, 11 + depth)).to(dev))
        lt.lt_map_set_norm(m, norms[0], norms[1], norms[2].reshape(-1), norms[3].reshape(-1))
        nets[name] = (m, lt.workspace(m, batch))
    n_pool = pool_np["x"].shape[0]
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        lo = ((k - 1) * batch) % (n_pool - batch + 1)
        rb = {f: v[lo:lo + batch] for f, v in pool.items()}
        tb = {"valid": ex["mask"][lo:lo + batch].reshape(1, -1)}
        for f in ("x", "y", "dx", "dy", "throughput"):
            tb[f] = ex[f][lo:lo + batch].reshape(1, -1)
        lr = 2e-3 * (0.5 ** (k / max(1, steps / 4)))
        m, ws = nets["classifier"]
        lt.lt_map_train_step(m, rb, tb, {"lr": lr, "step": k, "w_bce": 1.0, "w_l2": 0.0}, ws)
        m, ws = nets["regressor"]
        lt.lt_map_train_step(m, rb, tb, {"lr": lr, "step": k, "w_bce": 0.0, "w_l2": 1.0, "w_cos": w_cos}, ws)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    cls, reg = nets["classifier"][0], nets["regressor"][0]
    n = rays["x"].numel()
    stream = torch.cuda.current_stream()
    out = lt.empty_map_out(1, n, dev)

    def pair(dt, k=n):
        sub = rays if k == n else {f: v[:k] for f, v in rays.items()}
        o = out if k == n else lt.empty_map_out(1, k, dev)
        lt.lt_map_eval_ex(cls, dt, sub, o, k, lt.LT_EVAL_MASK_ONLY, None, stream)
        lt.lt_map_eval_ex(reg, dt, sub, o, k, lt.LT_EVAL_GATED, o["mask"], stream)
        return o
    res = {"classifier": "2 x 32 tanh, BCE", "regressor": f"5 x 32 tanh, MSE(x, y, I) + {w_cos:g} x (1 - cos)",
           "fit_steps": steps, "fit_seconds": t_fit,
           "flops_per_ray": map_flops_per_ray(32, 2, 1) + map_flops_per_ray(32, 5, 1)}
    # the regressor on the classifier's valid rays only (lt_mask_index +
    # lt_map_eval_indexed): the same values as the gated regressor on those
    # rays (tests/test_gpu_map_indexed.py), work in proportion to them
    cls_out = {"logit": torch.empty((1, n), dtype=torch.float32, device=dev),
               "mask": torch.empty((1, n), dtype=torch.uint8, device=dev)}
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    reg_out = {f: torch.empty((1, n), dtype=torch.float32, device=dev)
               for f in ("x", "y", "dx", "dy", "dz", "throughput")}

    def pair_indexed(dt):
        lt.lt_map_eval_ex(cls, dt, rays, cls_out, n, lt.LT_EVAL_MASK_ONLY, None, stream)
        lt.lt_mask_index(cls_out["mask"], n=n, capacity=n, idx=idx, count=cnt, stream=stream)
        lt.lt_map_eval_indexed(reg, dt, rays, idx, cnt, n, reg_out, stream)

    for name, dt in (("f32", lt.LT_F32), ("bf16", lt.LT_BF16)):
        t = time_kernel(lambda: pair(dt), stream, 5)
        res[f"{name}_ms"] = t * 1e3
        res[f"{name}_mrays_s"] = n / t / 1e6
        t_ix = time_kernel(lambda: pair_indexed(dt), stream, 5)
        res[f"{name}_indexed_ms"] = t_ix * 1e3
        res[f"{name}_indexed_mrays_s"] = n / t_ix / 1e6
        k = 65536
        g = eval_host(pair(dt, k))
        o = {f: v.cpu().numpy() for f, v in lt.lt_trace(h, (0, 0, 0), {f: v[:k] for f, v in rays.items()}).items()}
        res[f"{name}_error_vs_gpu_tracer"] = exit_error(g, o, k)
    torch.cuda.synchronize()
    res["indexed_valid_fraction"] = int(cnt.item()) / n
    res["indexed"] = ("classifier (LT_EVAL_MASK_ONLY), lt_mask_index, regressor on the listed rays "
                      "(lt_map_eval_indexed); its values equal the gated pair's on the valid rays")
    return res


def paper_recipe(lt, synth, dev, path=(1, 2, 10), n_valid=81_000_000, epochs=40, batch=8192,
                 uniform_steps=3000, n_eval=1 << 20, seed=3301, w_cos=200.0):
    """The paper's training recipe (Sec. 5.1) against the library's default
    short fit for one ghost path of the 11-surface lens, at the paper's network size
    (classifier 2 x 32, BCE; regressor 5 x 32, MSE + cosine direction loss):
    - paper: the regressor on n_valid rays (81 M by default, the paper's
      count per path) uniform over the path's valid region from the
      Markov-chain sampler (CIE wavelengths), the classifier
      on those plus as many invalid uniform rays (balanced), both for
      `epochs` epochs of `batch` rays with lr 1e-4 x 0.95 per 10,000 batches;
    - uniform: both on uniform rays (valid ones only count in the regression
      loss), uniform_steps steps of 65,536 with lr 2e-3 halved every quarter.
    Both are evaluated on n_eval uniform rays of the benchmark distribution
    against the GPU tracer."""
    import numpy as np
    import torch
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    data = F.sampler_dataset(h, path, n_valid, seed)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    reg_np = torch.stack([data["reg_exit"][k] for k in F.REG_FIELDS], 1).double().cpu().numpy()
    cls_np = {k: v.cpu().numpy() for k, v in data["cls_rays"].items()}
    reg_rays_np = {k: v.cpu().numpy() for k, v in data["reg_rays"].items()}
    norms_cls = F.map_norms(cls_np, [(np.ones(1, bool), np.zeros((1, 5)))])
    norms_reg = F.map_norms(reg_rays_np, [(np.ones(len(reg_np), bool), reg_np)])
    ev = lt.lt_rays_generate(h, n_eval, seed + 7)
    ev_t = {k: v.cpu().numpy() for k, v in lt.lt_trace(h, path, ev).items()}

    def new_nets():
        nets = {}
        for name, depth, norms in (("classifier", 2, norms_cls), ("regressor", 5, norms_reg)):
            m = lt.lt_map_create(32, depth, 1, lt.LT_ACT_TANH)
            lt.lt_map_set_params(m, torch.from_numpy(F.init_params(32, depth, 1, 11 + depth)).to(dev))
            lt.lt_map_set_norm(m, norms[0], norms[1], norms[2].reshape(-1), norms[3].reshape(-1))
            nets[name] = m
        return nets

    def evaluate(nets):
        o = lt.empty_map_out(1, n_eval, dev)
        lt.lt_map_eval_ex(nets["classifier"], lt.LT_F32, ev, o, n_eval, lt.LT_EVAL_MASK_ONLY, None, stream)
        lt.lt_map_eval_ex(nets["regressor"], lt.LT_F32, ev, o, n_eval, lt.LT_EVAL_GATED, o["mask"], stream)
        return exit_error(eval_host(o), ev_t, n_eval)

    # the paper's recipe
    nets = new_nets()
    zeros = torch.zeros((1, 2 * n_valid), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    tc = {"valid": data["cls_valid"].reshape(1, -1)}
    for k in F.REG_FIELDS:
        tc[k] = zeros
    steps_c, loss_c = F.fit_epochs(nets["classifier"], data["cls_rays"], tc, epochs, batch,
                                   {"w_bce": 1.0, "w_l2": 0.0}, seed + 3, stream=stream, graph_steps=512)
    tr = {"valid": torch.ones((1, n_valid), dtype=torch.uint8, device=dev)}
    for k in F.REG_FIELDS:
        tr[k] = data["reg_exit"][k].reshape(1, -1)
    steps_r, loss_r = F.fit_epochs(nets["regressor"], data["reg_rays"], tr, epochs, batch,
                                   {"w_bce": 0.0, "w_l2": 1.0, "w_cos": w_cos}, seed + 4, stream=stream,
                                   graph_steps=512)
    torch.cuda.synchronize()
    t_paper = time.perf_counter() - t0
    err_paper = evaluate(nets)
    # the default recipe: uniform rays, short schedule
    nets_u = new_nets()
    pool = lt.lt_rays_generate(h, 1 << 22, seed + 5)
    pex = lt.lt_trace(h, path, pool)
    wsc = lt.workspace(nets_u["classifier"], 65536)
    wsr = lt.workspace(nets_u["regressor"], 65536)
    t0 = time.perf_counter()
    for k in range(1, uniform_steps + 1):
        lo = ((k - 1) * 65536) % ((1 << 22) - 65536 + 1)
        rb = {f: v[lo:lo + 65536] for f, v in pool.items()}
        tb = {"valid": pex["mask"][lo:lo + 65536].reshape(1, -1)}
        for f in F.REG_FIELDS:
            tb[f] = pex[f][lo:lo + 65536].reshape(1, -1)
        lr = 2e-3 * (0.5 ** (k / max(1, uniform_steps / 4)))
        lt.lt_map_train_step(nets_u["classifier"], rb, tb, {"lr": lr, "step": k, "w_bce": 1.0, "w_l2": 0.0}, wsc)
        lt.lt_map_train_step(nets_u["regressor"], rb, tb,
                             {"lr": lr, "step": k, "w_bce": 0.0, "w_l2": 1.0, "w_cos": w_cos}, wsr)
    torch.cuda.synchronize()
    t_uniform = time.perf_counter() - t0
    err_uniform = evaluate(nets_u)
    res = {"path": list(path), "lens": "11-surface double-Gauss-style lens",
           "uniform_valid_fraction": float(ev_t["mask"].mean()),
           "networks": "classifier 2 x 32 tanh (BCE), regressor 5 x 32 tanh "
                       f"(MSE on x, y, I + {w_cos:g} x (1 - cos) on direction), FP32 evaluation",
           "paper_recipe": {"data": f"{n_valid} valid rays from the Markov-chain sampler (CIE wavelengths) "
                                    f"for the regressor; those + {n_valid} invalid uniform rays for the "
                                    "classifier",
                            "schedule": f"{epochs} epochs, batch {batch}, lr 1e-4 x 0.95 per 10,000 batches",
                            "steps_run_as": "recorded runs of 512 steps (fit.TrainGraph), the rest of each epoch eager",
                            "classifier_steps": steps_c, "regressor_steps": steps_r,
                            "data_seconds": t_data, "fit_seconds": t_paper,
                            "chain_steps": int(data["chain_steps"]), "uniform_rays_traced": int(data["uniform_rays"]),
                            "final_loss": {"classifier": float(loss_c[0]), "regressor": float(loss_r[0])},
                            "error_vs_gpu_tracer": err_paper},
           "uniform_recipe": {"data": "uniform rays (4,194,304-ray pool), labelled by the tracer",
                              "schedule": f"{uniform_steps} steps of 65,536, lr 2e-3 halved every quarter",
                              "fit_seconds": t_uniform, "error_vs_gpu_tracer": err_uniform},
           "eval": f"{n_eval} uniform rays of the benchmark distribution"}
    del data, pool, pex, ev
    torch.cuda.empty_cache()
    return res


def serving(lt, synth, dev, n_req=20000, loads=(0.5, 0.8), seed=5005, ring_rays=1 << 27):
    """Serving run: 8 lenses (4..22 surfaces) with resident maps; Poisson
    arrivals of 1k..1M-ray requests (log-uniform); memory-admitted
    continuous batching on 8 streams by the native request loop
    (lt_server_*), requests split into chunks of 262,144 rays.  Offered load
    relative to the saturated rate measured with all requests queued at
    t = 0.  The Python loop's saturated rate (the same policy in Python over
    per-chunk wrapper calls, on the first 2,000 requests) is reported beside
    the native one.  Request outputs are views into a ring of ring_rays rays
    per field: admission holds at most mem_budget / bytes_per_ray = 67 M rays
    in flight, so a ring of 134 M never hands an in-flight request's range to
    a new one (outputs are not read here; the serving tests check them)."""
    import numpy as np
    import torch
    from paper_2605_04017_amd.serve import (GpuExecutor, NativeScheduler, Scheduler, latency_stats,
                                            poisson_requests, run_trace)
    lenses = synth.serve_lenses()
    hl, maps, pools = [], [], []
    for i, L in enumerate(lenses):
        hl.append(lt.lt_lens_create(L.surfaces, L.glasses))
        pools.append({k: torch.from_numpy(v).to(dev) for k, v in synth.make_rays(L, 1000000, 7000 + i).items()})
        mm = lt.lt_map_create(MAP_WIDTH, MAP_DEPTH, 1)
        lt.lt_map_set_params(mm, torch.from_numpy(F.init_params(MAP_WIDTH, MAP_DEPTH, 1, 80 + i)).to(dev))
        maps.append(mm)
    res = {}

    def requests(rate):
        reqs = poisson_requests(n_req, rate, 8, seed)
        for r in reqs:
            off = (r.rid * 7919) % (1000000 - r.n + 1)
            r.payload = {k: v[off:off + r.n] for k, v in pools[r.lens].items()}
        return reqs

    for mode, dtype in (("map", lt.LT_BF16), ("map", lt.LT_F32), ("trace", 0)):
        key = f"{mode}_{'bf16' if (mode == 'map' and dtype == lt.LT_BF16) else 'f32'}"
        if mode == "map":
            for m in maps:
                lt.lt_map_quantize(m, dtype)
        sizes = [r.n for r in poisson_requests(n_req, 1.0, 8, seed)]

        ring = lt.empty_map_out(1, ring_rays, dev) if mode == "map" else lt.empty_exit(ring_rays, dev)

        def run(rate):
            reqs = requests(rate)
            pos = 0
            for r in reqs:
                if pos + r.n > ring_rays:
                    pos = 0
                out = {k: (v[:, pos:pos + r.n] if v.dim() == 2 else v[pos:pos + r.n]) for k, v in ring.items()}
                pos += r.n
                r.payload = (r.payload, out)
            torch.cuda.synchronize()
            for r in reqs:   # marshalled up front, as a client builds its requests
                rays, out = r.payload
                r.prepared = (lt.Server.prepare_map(maps[r.lens], dtype, rays, out, r.n) if mode == "map"
                              else lt.Server.prepare_trace(hl[r.lens], (0, 0, 0), rays, out, r.n))
            srv = lt.Server(8, chunk=262144, mem_budget=4 << 30, bytes_per_ray=64)
            sched = NativeScheduler(srv, hl, maps, mode, dtype)
            done = run_trace(sched, reqs, sched.clock)
            torch.cuda.synchronize()
            srv.close()
            span = max(r.done for r in done) - min(r.arrival for r in done)
            return done, sum(r.n for r in done) / span

        _, sat = run(1e9)  # everything queued at once
        out = {"saturated_mrays_s": sat / 1e6}
        for rho in loads:
            rate = rho * sat / float(np.mean(sizes))
            done, thr = run(rate)
            st = latency_stats(done)
            out[f"load_{rho}"] = {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                                  "mrays_s": thr / 1e6, "requests": st["n"]}
        del ring
        if key == "map_bf16":
            reqs = requests(1e9)[:2000]
            ex = GpuExecutor(8, hl, maps, mode, dtype)
            sched = Scheduler(ex, mem_budget_bytes=4 << 30, bytes_per_ray=64, chunk=262144)
            ex.start_clock()
            done = run_trace(sched, reqs, ex.clock)
            torch.cuda.synchronize()
            span = max(r.done for r in done) - min(r.arrival for r in done)
            out["python_loop_saturated_mrays_s"] = sum(r.n for r in done) / span / 1e6
        res[key] = out
    res["loop"] = "native (lt_server_*), 8 streams, chunks of 262,144 rays, 4 GiB admission budget"
    return res


def train_epoch(lt, synth, dev, n_total=67108864, batch=65536, seed=4004):
    """One training epoch of the 5 x 128 map on the training workload: the
    67,108,864 rays are drawn on the device (lt_rays_generate), labelled by
    the FP32 tracer (transmit path), and consumed in 1,024 steps of 65,536
    (lt_map_train_step: forward, BCE + masked L2, backward, Adam).  Times are
    HIP events on the stream; the wall time of the step loop (Python call
    overhead included) is reported beside them."""
    import numpy as np
    import torch
    lens = synth.config_lens(4)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    rays = lt.lt_rays_generate(h, n_total, seed, stream=stream)
    ev[1].record(stream)
    ex = lt.lt_trace(h, (0, 0, 0), rays, None, n_total, stream)
    ev[2].record(stream)
    torch.cuda.synchronize()
    t_gen = ev[0].elapsed_time(ev[1]) * 1e-3
    t_trace = ev[1].elapsed_time(ev[2]) * 1e-3
    tgt = {"valid": ex["mask"].reshape(1, -1)}
    for f in ("x", "y", "dx", "dy", "throughput"):
        tgt[f] = ex[f].reshape(1, -1)
    # normalisation from the first batch (inputs) and its valid rays (outputs)
    first = {k: rays[k][:batch].cpu().numpy() for k in synth.RAY_FIELDS}
    ok = ex["mask"][:batch].bool()
    reg = torch.stack([ex[k][:batch][ok] for k in ("x", "y", "dx", "dy", "throughput")], 1).double()
    norms = F.map_norms(first, [(ok.cpu().numpy(), reg.cpu().numpy())])
    m = lt.lt_map_create(MAP_WIDTH, MAP_DEPTH, 1, lt.LT_ACT_TANH)
    lt.lt_map_set_params(m, torch.from_numpy(F.init_params(MAP_WIDTH, MAP_DEPTH, 1, 6)).to(dev))
    lt.lt_map_set_norm(m, norms[0], norms[1], norms[2].reshape(-1), norms[3].reshape(-1))
    ws = lt.workspace(m, batch)
    loss = torch.zeros(3, dtype=torch.float32, device=dev)
    steps = n_total // batch
    batches = []
    for k in range(steps):
        lo, hi = k * batch, (k + 1) * batch
        batches.append(({f: v[lo:hi] for f, v in rays.items()},
                        {f: v[:, lo:hi] for f, v in tgt.items()}))
    torch.cuda.synchronize()
    first_loss = None
    w0 = time.perf_counter()
    ev[2].record(stream)
    for k, (rb, tb) in enumerate(batches, 1):
        lr = 2e-3 * (0.5 ** (k / (steps / 4)))
        lt.lt_map_train_step(m, rb, tb, {"lr": lr, "step": k, "w_bce": 1.0, "w_l2": 4.0}, ws, loss,
                             batch, stream)
        if k == 1:
            first_loss = loss.clone()
    ev[3].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    t_train = ev[2].elapsed_time(ev[3]) * 1e-3
    # the same steps as recorded runs of 64 (fit.TrainGraph) on a twin map:
    # per run, the run's 64 batches are copied into the graph's buffers, the
    # 64 schedule entries written with one copy, and the graph replayed
    g_map = lt.lt_map_create(MAP_WIDTH, MAP_DEPTH, 1, lt.LT_ACT_TANH)
    lt.lt_map_set_params(g_map, torch.from_numpy(F.init_params(MAP_WIDTH, MAP_DEPTH, 1, 6)).to(dev))
    lt.lt_map_set_norm(g_map, norms[0], norms[1], norms[2].reshape(-1), norms[3].reshape(-1))
    K = 64
    t_rec = time.perf_counter()
    graph = F.TrainGraph(g_map, K, batch, {"w_bce": 1.0, "w_l2": 4.0}, dev)
    t_rec = time.perf_counter() - t_rec
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    ev[2].record(stream)
    for r0 in range(0, steps, K):
        lo, hi = r0 * batch, (r0 + K) * batch
        for f, v in graph.rays.items():
            v.copy_(rays[f][lo:hi])
        for f, v in graph.targets.items():
            v.copy_(tgt[f][:, lo:hi].reshape(1, K, batch).permute(1, 0, 2))
        graph.run([2e-3 * (0.5 ** (k / (steps / 4))) for k in range(r0 + 1, r0 + K + 1)], r0 + 1)
    ev[3].record(stream)
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - w1
    t_graph = ev[2].elapsed_time(ev[3]) * 1e-3
    same = bool(torch.equal(lt.lt_map_get_params(g_map), lt.lt_map_get_params(m)))
    # replays alone (data already in place): the steps' own device time
    ev[2].record(stream)
    for rep in range(4):
        graph.run([1e-4] * K, steps + 1 + rep * K)
    ev[3].record(stream)
    torch.cuda.synchronize()
    t_replay = ev[2].elapsed_time(ev[3]) * 1e-3 / (4 * K)
    fpr = map_flops_per_ray()
    valid = float(ex["mask"].float().mean())
    del batches, rays, ex, tgt, ws, graph
    torch.cuda.empty_cache()
    return {"rays": n_total, "batch": batch, "steps": steps,
            "generate_ms": t_gen * 1e3, "trace_ms": t_trace * 1e3, "train_ms": t_train * 1e3,
            "step_ms": t_train / steps * 1e3, "train_wall_s": wall,
            "graph": {"steps_per_run": K, "record_s": t_rec, "train_ms_with_batch_copies": t_graph * 1e3,
                      "train_wall_s": wall_graph, "step_ms": t_graph / steps * 1e3,
                      "step_ms_replay_only": t_replay * 1e3, "params_identical_to_eager": same},
            "train_mrays_s": n_total / t_train / 1e6,
            "train_tflops_3x_forward": 3 * fpr * n_total / t_train / 1e12,
            "valid_fraction": valid,
            "loss_first_step": [float(v) for v in first_loss.cpu()],
            "loss_last_step": [float(v) for v in loss.cpu()]}


def fit_multi_head(lt, synth, lens, h, paths, dev, steps, n_pool=1 << 21, batch=65536, seed=3004):
    """One 5 x 128 trunk with a head per path (canonical input), fitted for
    `steps` steps on GPU traces of every path."""
    import numpy as np
    import torch
    P = len(paths)
    pool_np = synth.make_rays(lens, n_pool, seed)
    pool = {k: torch.from_numpy(v).to(dev) for k, v in pool_np.items()}
    tgt = {"valid": torch.empty((P, n_pool), dtype=torch.uint8, device=dev)}
    for f in ("x", "y", "dx", "dy", "throughput"):
        tgt[f] = torch.empty((P, n_pool), dtype=torch.float32, device=dev)
    ex = lt.empty_exit(n_pool, dev)
    targets = []
    for k, p in enumerate(paths):
        lt.lt_trace(h, p, pool, ex, n_pool)
        tgt["valid"][k].copy_(ex["mask"])
        for f in ("x", "y", "dx", "dy", "throughput"):
            tgt[f][k].copy_(ex[f])
        ok = ex["mask"].bool()
        targets.append((ok.cpu().numpy(), torch.stack([ex[f][ok] for f in ("x", "y", "dx", "dy", "throughput")],
                                                       1).double().cpu().numpy()))
    norms = F.map_norms(pool_np, targets, canonical=True)
    m = lt.lt_map_create(MAP_WIDTH, MAP_DEPTH, P, lt.LT_ACT_TANH, True)
    lt.lt_map_set_params(m, torch.from_numpy(F.init_params(MAP_WIDTH, MAP_DEPTH, P, 9)).to(dev))
    lt.lt_map_set_norm(m, norms[0], norms[1], norms[2].reshape(-1), norms[3].reshape(-1))
    ws = lt.workspace(m, batch)
    t0 = time.perf_counter()
    loss = None
    for k in range(1, steps + 1):
        lo = ((k - 1) * batch) % (n_pool - batch + 1)
        rb = {f: v[lo:lo + batch] for f, v in pool.items()}
        tb = {f: v[:, lo:lo + batch].contiguous() for f, v in tgt.items()}
        lr = 2e-3 * (0.5 ** (k / max(1, steps / 4)))
        loss = lt.lt_map_train_step(m, rb, tb, {"lr": lr, "step": k, "w_bce": 1.0, "w_l2": 4.0}, ws)
    torch.cuda.synchronize()
    return m, time.perf_counter() - t0, [float(v) for v in loss.cpu()], norms


def multi_path_error(lt, h, m, paths, dtype, rays, n_sample=65536):
    """Map error over every (path, ray) pair of the first n_sample rays
    against the GPU tracer: mask agreement over all pairs, exit positions
    over the pairs valid in both; the transmit head on its own beside it."""
    import numpy as np
    sub = {k: v[:n_sample] for k, v in rays.items()}
    g = {k: v.cpu().numpy() for k, v in lt.lt_map_eval(m, dtype, sub).items()}
    agree, pos, ghost_p50, transmit = [], [], [], None
    for i, p in enumerate(paths):
        o = {k: v.cpu().numpy() for k, v in lt.lt_trace(h, p, sub).items()}
        gi = {k: v[i] for k, v in g.items()}
        e = exit_error(gi, o, n_sample)
        if i == 0:
            transmit = e
        elif "pos_mm_p50" in e:
            ghost_p50.append(e["pos_mm_p50"])
        both = gi["mask"].astype(bool) & o["mask"].astype(bool)
        agree.append(gi["mask"].astype(bool) == o["mask"].astype(bool))
        pos.append(np.hypot(gi["x"][both] - o["x"][both], gi["y"][both] - o["y"][both]))
    pos = np.concatenate(pos)
    return {"pairs": len(paths) * n_sample, "valid_pairs_in_both": int(pos.size),
            "mask_agreement": float(np.mean(np.concatenate(agree))),
            "pos_mm_p50": float(np.median(pos)), "pos_mm_p99": float(np.quantile(pos, 0.99)),
            "transmit": transmit,
            "ghost_pos_mm_p50_median_over_paths": float(np.median(ghost_p50)) if ghost_p50 else None}


def all_paths_paths(lens):
    nr = lens.n_refracting
    return [(0, 0, 0)] + [(1, j, i) for j in range(1, nr + 1) for i in range(j + 1, nr + 1)]


def map_compact_bytes(n, heads, counts, with_dz=True):
    """Algorithmic HBM bytes of one compacted map launch: 24 B of input per
    ray, the mask bitmap (one bit per ray and head, in 32-bit words) and 24 B
    (28 with dz) per valid ray-path: index, x, y, dx, dy, (dz), throughput."""
    return 24 * n + 4 * heads * ((n + 31) // 32) + (28 if with_dz else 24) * int(sum(counts))


def all_paths(lt, synth, dev, args):
    """The headline workload: 16,777,216 rays of the 11-surface lens, every
    path with at most two reflections (transmit + 55 ghosts).  Tracer: one
    launch per path.  Map: one 5 x 128 trunk with 56 heads (canonical
    input), fitted on GPU traces of all 56 paths.  The timed step runs the
    compacted tracer over all paths and the compacted FP32 map; the other
    precisions, uncompacted outputs and tracer variants are timed beside it."""
    import numpy as np
    import torch
    n = args.rays_all
    lens = synth.config_lens(3)
    rays_np = synth.config_rays(3, n)
    rays = {k: torch.from_numpy(v).to(dev) for k, v in rays_np.items()}
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    paths = all_paths_paths(lens)
    P = len(paths)
    stream = torch.cuda.current_stream()

    # tracer outputs: compacted, one buffer set reused by every path launch
    cout = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in lt.EXIT_FIELDS[1:]}
    cidx = torch.empty(n, dtype=torch.int64, device=dev)
    tcounts = torch.empty(P, dtype=torch.int64, device=dev)

    def trace_all_compact(flags=0):
        for k, p in enumerate(paths):
            lt.lt_trace_compact(h, p, rays, cout, cidx, tcounts[k:k + 1], n, flags, stream)

    # the map, fitted on GPU traces of every path
    m, t_fit, fit_loss, norms = fit_multi_head(lt, synth, lens, h, paths, dev, args.fit_steps)
    flat = lt.lt_map_get_params(m).cpu().numpy()
    for dt in (lt.LT_F32, lt.LT_BF16, lt.LT_FP8):
        lt.lt_map_quantize(m, dt)
    # compacted map outputs: capacity = the largest head count, with margin
    probe = lt.lt_map_eval_compact(m, lt.LT_F32, rays, capacity=n // 4, with_bits=False)
    cap = int(probe["count"].max()) * 9 // 8 + 1024
    del probe
    torch.cuda.empty_cache()
    cmp = lt.lt_map_eval_compact(m, lt.LT_F32, rays, capacity=cap)
    torch.cuda.synchronize()
    print(f"# all paths: map fitted in {t_fit:.1f} s, compacted capacity {cap}", file=sys.stderr, flush=True)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        trace_all_compact()
        if ev is not None:
            ev[1].record(stream)
        lt.lt_map_eval_compact(m, lt.LT_F32, rays, capacity=cap, out=cmp, n=n, stream=stream)
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
    t_trace = float(np.mean([e[0].elapsed_time(e[1]) for e in evs])) * 1e-3
    t_map = float(np.mean([e[1].elapsed_time(e[2]) for e in evs])) * 1e-3
    counts_f32 = cmp["count"].cpu().numpy()
    assert counts_f32.max() <= cap, "compacted map output overflowed its capacity"
    tvalid = tcounts.cpu().numpy()
    print(f"# all paths: timed {args.steps} steps", file=sys.stderr, flush=True)

    # other precisions and uncompacted outputs of the map
    reps = 3
    t_cmp, cnt = {"f32": t_map}, {"f32": counts_f32}
    for name, dt in (("bf16", lt.LT_BF16), ("fp8", lt.LT_FP8)):
        t_cmp[name] = time_kernel(lambda: lt.lt_map_eval_compact(m, dt, rays, capacity=cap, out=cmp, n=n,
                                                                  stream=stream), stream, reps)
        cnt[name] = cmp["count"].cpu().numpy()
        assert cnt[name].max() <= cap, "compacted map output overflowed its capacity"
    mout = lt.empty_map_out(P, n, dev)
    t_full = {}
    for name, dt in (("f32", lt.LT_F32), ("bf16", lt.LT_BF16), ("fp8", lt.LT_FP8)):
        t_full[name] = time_kernel(lambda: lt.lt_map_eval(m, dt, rays, mout, n, stream), stream, 2)
    del mout
    torch.cuda.empty_cache()
    # tracer variants: uncompacted default, compacted FP64 option, compacted plain FP32
    out = lt.empty_exit(n, dev)

    def trace_all(flags=0):
        for p in paths:
            lt.lt_trace_ex(h, p, rays, out, n, flags, stream)
    t_trace_full = time_kernel(trace_all, stream, 1)
    t_trace_f64 = time_kernel(lambda: trace_all_compact(lt.LT_TRACE_FP64), stream, 1)
    t_trace_plain = time_kernel(lambda: trace_all_compact(lt.LT_TRACE_PLAIN_FP32), stream, 1)
    del out
    print("# all paths: variants timed", file=sys.stderr, flush=True)

    errors = {name: multi_path_error(lt, h, m, paths, dt, rays)
              for name, dt in (("f32", lt.LT_F32), ("bf16", lt.LT_BF16), ("fp8", lt.LT_FP8))}
    fpr = map_flops_per_ray(heads=P)
    tracers = {"float_pair_compact": t_trace, "float_pair": t_trace_full, "fp64_option_compact": t_trace_f64}
    res = {"paths": P, "rays": n, "ray_paths": P * n,
           "trace_ms": {"float_pair_compact": t_trace * 1e3, "float_pair": t_trace_full * 1e3,
                        "fp64_option_compact": t_trace_f64 * 1e3,
                        "plain_fp32_compact_outside_tolerance": t_trace_plain * 1e3},
           "trace_mray_paths_s": {k: P * n / v / 1e6 for k, v in tracers.items()},
           "valid_fraction_transmit": float(tvalid[0]) / n,
           "valid_fraction_ghost_mean": float(tvalid[1:].mean()) / n,
           "map_compact_ms": {k: v * 1e3 for k, v in t_cmp.items()},
           "map_uncompacted_ms": {k: v * 1e3 for k, v in t_full.items()},
           "map_compact_mray_paths_s": {k: P * n / v / 1e6 for k, v in t_cmp.items()},
           "map_over_trace": {k: {tn: tt / v for tn, tt in tracers.items()} for k, v in t_cmp.items()},
           "map_valid_fraction": {k: float(v.sum()) / (P * n) for k, v in cnt.items()},
           "compact_capacity_per_head": cap,
           "fit": {"steps": args.fit_steps, "batch": 65536, "seconds": t_fit, "final_loss": fit_loss,
                   "map": "5 x 128 tanh, 56 heads, canonical input"},
           "map_error_vs_gpu_tracer": errors}
    rl = {}
    for name, peak in (("f32", MI355X_FP32_MFMA_TFLOPS), ("bf16", MI355X_BF16_MFMA_TFLOPS),
                       ("fp8", MI355X_FP8_MFMA_TFLOPS)):
        tf = fpr * n / t_cmp[name] / 1e12
        byt = map_compact_bytes(n, P, cnt[name])
        gbs = byt / t_cmp[name] / 1e9
        rl[name] = {"bound": "mfma", "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
                    "flops_per_ray": fpr, "algorithmic_bytes": byt, "hbm_gbs": gbs,
                    "hbm_frac": gbs / MI355X_HBM_GBS}
    res["roofline_by_dtype"] = rl
    res["wall_s_timed"] = wall
    res["_cpu"] = (flat, norms, rays_np, lens, paths)
    res["_t"] = (t_trace, t_map, wall)
    del rays, cout, cidx, cmp
    torch.cuda.empty_cache()
    return res


FLARE_SENSOR = (36.0, 24.0, 720, 480)
FLARE_BANDS = ((600.0, 700.0), (500.0, 600.0), (400.0, 500.0))   # R, G, B


def flare(lt, synth, dev, steps=10000, n_render=1 << 20, theta_deg=10.0, n_ghosts=8,
          batch=65536, seed=6006, n_pool=1 << 22):
    """Forward light tracing of a distant point light (Sec. 3 flare sum; the
    forward half of the rendering pipeline, whose transmit image comes from
    backward path tracing): per RGB channel, 1,048,576 rays from the light
    at theta_deg off axis, p_in uniform on the first surface's clear
    aperture in the forward input plane, wavelength uniform in the channel's
    band, through the n_ghosts brightest two-reflection ghosts of the
    11-surface lens, splatted into per-path 720 x 480 images of the
    36 x 24 mm sensor.

    Map: one forward map (5 x 128 tanh trunk, one head per ghost, canonical
    input), fitted for `steps` steps on GPU forward traces of rays from
    directions within 15 degrees of the axis (so it serves any light in that
    cone).  Frame time: map (BF16) + splat versus forward trace + splat, on
    the same resident rays.  Image error: relative L1 of each path's map
    image against its traced image, at the pixel size and after 4 x 4 and
    16 x 16 binning, next to the Monte Carlo floor (two traced renders with
    independent rays)."""
    import math
    import numpy as np
    import torch
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    stream = torch.cuda.current_stream()
    nr = lens.n_refracting
    ghosts = [(1, j, i) for j in range(1, nr + 1) for i in range(j + 1, nr + 1)]
    th = math.radians(theta_deg)
    light = (math.sin(th), 0.0, math.cos(th))
    W, H, NX, NY = FLARE_SENSOR
    fwd = lt.LT_TRACE_FORWARD

    # the brightest ghosts of this light (green band)
    n_probe = 1 << 18
    probe = lt.lt_rays_generate_forward(h, n_probe, seed, light, lam_range=FLARE_BANDS[1])
    energy = []
    for p in ghosts:
        o = lt.lt_trace_ex(h, p, probe, None, n_probe, fwd, stream)
        energy.append(float(lt.lt_splat(o["x"], o["y"], o["dz"], o["throughput"], FLARE_SENSOR,
                                        mask=o["mask"], stream=stream).sum()))
    order = np.argsort(energy)[::-1]
    paths = [ghosts[k] for k in order[:n_ghosts]]
    P = len(paths)
    covered = float(np.sum(np.asarray(energy)[order[:n_ghosts]]) / max(1e-30, np.sum(energy)))

    # training data: forward traces of a 15-degree cone of directions
    t0 = time.perf_counter()
    pool_np = synth.make_forward_rays(lens, n_pool, seed + 1, half_angle_deg=15.0, aperture_scale=1.0)
    pool = {k: torch.from_numpy(v).to(dev) for k, v in pool_np.items()}
    tgt = {"valid": torch.empty((P, n_pool), dtype=torch.uint8, device=dev)}
    for f in ("x", "y", "dx", "dy", "throughput"):
        tgt[f] = torch.empty((P, n_pool), dtype=torch.float32, device=dev)
    ex = lt.empty_exit(n_pool, dev)
    targets = []
    for k, p in enumerate(paths):
        lt.lt_trace_ex(h, p, pool, ex, n_pool, fwd, stream)
        tgt["valid"][k].copy_(ex["mask"])
        for f in ("x", "y", "dx", "dy", "throughput"):
            tgt[f][k].copy_(ex[f])
        ok = ex["mask"].bool().cpu().numpy()
        targets.append((ok, np.stack([ex[f].cpu().numpy()[ok].astype(np.float64)
                                      for f in ("x", "y", "dx", "dy", "throughput")], 1)))
    norms = F.map_norms(pool_np, targets, canonical=True)
    m = lt.lt_map_create(MAP_WIDTH, MAP_DEPTH, P, lt.LT_ACT_TANH, True, True)
    lt.lt_map_set_params(m, torch.from_numpy(F.init_params(MAP_WIDTH, MAP_DEPTH, P, 7)).to(dev))
    lt.lt_map_set_norm(m, norms[0], norms[1], norms[2].reshape(-1), norms[3].reshape(-1))
    ws = lt.workspace(m, batch)
    del ex
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss = None
    for k in range(1, steps + 1):
        lo = ((k - 1) * batch) % (n_pool - batch + 1)
        rb = {f: v[lo:lo + batch] for f, v in pool.items()}
        tb = {f: v[:, lo:lo + batch].contiguous() for f, v in tgt.items()}
        lr = 2e-3 * (0.5 ** (k / max(1, steps / 4)))
        loss = lt.lt_map_train_step(m, rb, tb, {"lr": lr, "step": k, "w_bce": 1.0, "w_l2": 4.0}, ws)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    del pool, tgt, ws

    # one frame: three channels, every path
    n = n_render
    rays = [lt.lt_rays_generate_forward(h, n, seed + 10 + ch, light, lam_range=b)
            for ch, b in enumerate(FLARE_BANDS)]
    rays2 = [lt.lt_rays_generate_forward(h, n, seed + 20 + ch, light, lam_range=b)
             for ch, b in enumerate(FLARE_BANDS)]
    img_map = torch.zeros((3, P, NY, NX), dtype=torch.float32, device=dev)
    img_tr = torch.zeros_like(img_map)
    img_tr2 = torch.zeros_like(img_map)
    mout = lt.empty_map_out(P, n, dev)
    eout = lt.empty_exit(n, dev)
    lt.lt_map_quantize(m, lt.LT_BF16, stream)

    def render_map(dt=lt.LT_BF16):
        img_map.zero_()
        for ch in range(3):
            lt.lt_map_eval(m, dt, rays[ch], mout, n, stream)
            lt.lt_splat(mout["x"], mout["y"], mout["dz"], mout["throughput"], FLARE_SENSOR,
                        images=img_map[ch], mask=mout["mask"], n=P * n, n_per_image=n,
                        scale=1.0 / n, stream=stream)

    def render_trace(rs=rays, img=img_tr):
        img.zero_()
        for ch in range(3):
            for k, p in enumerate(paths):
                lt.lt_trace_ex(h, p, rs[ch], eout, n, fwd, stream)
                lt.lt_splat(eout["x"], eout["y"], eout["dz"], eout["throughput"], FLARE_SENSOR,
                            images=img[ch, k], mask=eout["mask"], n=n, scale=1.0 / n, stream=stream)
    t_map = time_kernel(render_map, stream, 5)
    t_tr = time_kernel(render_trace, stream, 3)
    render_trace(rays2, img_tr2)
    t_eval = time_kernel(lambda: lt.lt_map_eval(m, lt.LT_BF16, rays[1], mout, n, stream), stream, 5)
    t_splat = time_kernel(lambda: lt.lt_splat(mout["x"], mout["y"], mout["dz"], mout["throughput"],
                                              FLARE_SENSOR, images=img_map[1], mask=mout["mask"],
                                              n=P * n, n_per_image=n, scale=1.0 / n, stream=stream),
                          stream, 10)
    render_map()
    torch.cuda.synchronize()

    def rel_l1(a, b, binning=1):
        if binning > 1:
            pool = torch.nn.functional.avg_pool2d
            a, b = (pool(t.reshape(-1, 1, NY, NX), binning) for t in (a, b))
        return float((a - b).abs().sum() / b.abs().sum().clamp_min(1e-30))

    def errs(a, b, c):
        return {f"rel_l1_{tag}": rel_l1(a, b, bn) for tag, bn in (("px", 1), ("4x4", 4), ("16x16", 16))} | {
            f"mc_floor_{tag}": rel_l1(c, b, bn) for tag, bn in (("px", 1), ("4x4", 4), ("16x16", 16))}
    per_path = {}
    for k, p in enumerate(paths):
        per_path[f"ghost{p[1]},{p[2]}"] = {"energy_share": float(img_tr[:, k].sum() / img_tr.sum()),
                                           **errs(img_map[:, k], img_tr[:, k], img_tr2[:, k])}
    splat_bytes = 17 * P * n
    res = {"lens": "11-surface double-Gauss-style lens", "light": f"point at infinity, {theta_deg} deg",
           "rays_per_channel": n, "channels": "RGB bands 600-700 / 500-600 / 400-500 nm",
           "sensor": {"mm": [W, H], "pixels": [NX, NY]},
           "paths": P, "selected_ghosts_energy_share_of_all_55": covered,
           "map": f"5 x {MAP_WIDTH} tanh, {P} heads, canonical input, forward exits, BF16 eval",
           "fit_steps": steps, "fit_seconds": t_fit, "fit_data_seconds": t_data,
           "fit_final_loss": [float(v) for v in loss.cpu()],
           "frame_ms_map_bf16": t_map * 1e3, "frame_ms_trace": t_tr * 1e3,
           "frame_speedup_map_over_trace": t_tr / t_map,
           "ray_paths_per_s_map_G": 3 * n * P / t_map / 1e9,
           "ray_paths_per_s_trace_G": 3 * n * P / t_tr / 1e9,
           "map_eval_ms_per_channel": t_eval * 1e3, "splat_ms_per_channel": t_splat * 1e3,
           "splat_roofline": {"bound": "hbm", "achieved": splat_bytes / t_splat / 1e9,
                              "peak": MI355X_HBM_GBS, "unit": "GB/s",
                              "frac": splat_bytes / t_splat / 1e9 / MI355X_HBM_GBS,
                              "bytes_per_ray": 17, "rays_per_launch": P * n},
           "flare_image": errs(img_map.sum(1), img_tr.sum(1), img_tr2.sum(1)),
           "per_path": per_path}
    del img_map, img_tr, img_tr2, mout, eout, rays, rays2
    torch.cuda.empty_cache()
    return res


def sampler_yield(lt, synth, dev, path=(1, 2, 10), n_chains=1 << 20, steps=32, burn_in=256,
                  n_uniform=1 << 24, seed=7007):
    """Training-data generation for one ghost path of the 11-surface lens
    with a small valid region (Sec. 5.1: a Markov chain with a binary
    visibility target raises the valid-sample yield): valid labelled rays
    per second from the device chains (1,048,576 chains, 32 timed steps after
    a 256-step burn-in) against rejection sampling (16,777,216 uniform rays
    traced with compacted output).  The chains' outputs repeat a state when
    a proposal is rejected, so the rate of distinct valid samples (accepted
    proposals) is reported too."""
    import numpy as np
    import torch
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    stream = torch.cuda.current_stream()
    uni = lt.lt_rays_generate(h, n_uniform, seed)
    cout = {k: torch.empty(n_uniform, dtype=torch.float32, device=dev) for k in lt.EXIT_FIELDS[1:]}
    cidx = torch.empty(n_uniform, dtype=torch.int64, device=dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)

    def rejection():
        lt.lt_rays_generate(h, n_uniform, seed, out=uni, stream=stream)
        lt.lt_trace_compact(h, path, uni, cout, cidx, cnt, n_uniform, 0, stream)
    t_rej = time_kernel(rejection, stream, 3)
    n_valid = int(cnt.item())
    del uni, cout, cidx
    st = lt.lt_mcmc_init(lt.mcmc_state(n_chains, dev), 0.05)
    rays = {k: torch.empty((steps, n_chains), dtype=torch.float32, device=dev) for k in lt.RAY_FIELDS}
    ex = {k: v.view(steps, n_chains) for k, v in lt.empty_exit(steps * n_chains, dev).items()}
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    first = 0
    for _ in range(burn_in // steps):
        lt.lt_mcmc_run(h, path, st, steps, seed, first, rays_out=rays, exit_out=ex, counts=counts,
                       stream=stream)
        first += steps
    torch.cuda.synchronize()
    c0 = counts.cpu().numpy().copy()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lt.lt_mcmc_run(h, path, st, steps, seed, first, rays_out=rays, exit_out=ex, counts=counts, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t_mc = e0.elapsed_time(e1) * 1e-3
    c1 = counts.cpu().numpy()
    d = (c1 - c0).astype(np.float64)
    valid_out = float(ex["mask"].float().sum())
    res = {"path": list(path), "lens": "11-surface double-Gauss-style lens",
           "uniform_valid_fraction": n_valid / n_uniform,
           "rejection_valid_rays_per_s_M": n_valid / t_rej / 1e6,
           "rejection_ms": t_rej * 1e3, "rejection_rays": n_uniform,
           "chains": n_chains, "steps_timed": steps, "burn_in_steps": burn_in,
           "mcmc_ms": t_mc * 1e3,
           "mcmc_valid_outputs_fraction": valid_out / (steps * n_chains),
           "mcmc_valid_rays_per_s_M": valid_out / t_mc / 1e6,
           "mcmc_distinct_valid_rays_per_s_M": (d[1] + d[3]) / t_mc / 1e6,
           "small_step_acceptance": d[3] / max(1.0, d[2]),
           "uniform_fraction_estimate_from_chains": c1[1] / max(1, c1[0]),
           "valid_rays_per_traced_ray": {"rejection": n_valid / n_uniform,
                                         "mcmc_outputs": valid_out / (steps * n_chains),
                                         "mcmc_distinct": (d[1] + d[3]) / (steps * n_chains)}}
    del rays, ex, st
    torch.cuda.empty_cache()
    return res


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "map_f32_c2_4M_traffic.md")
TRAFFIC_ALL_SUMMARY = os.path.join(ROOT, "profiles", "map_compact_56heads_16M_traffic.md")
MAP_F32_SOURCES = ("paper_2605_04017_amd/csrc/lt_map_f32.hip", "paper_2605_04017_amd/csrc/lt_map_dev.h",
                   "paper_2605_04017_amd/csrc/lt_map.h")
MAP_BF16_SOURCES = ("paper_2605_04017_amd/csrc/lt_map.hip",)
COPY_PROBE_BYTES = 512 << 20


def source_hash(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(summary, sources):
    """HBM bytes per launch of a map kernel from a committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by the counter's
    reading for a plain copy of known size), or None when the kernel sources
    changed since the counters were taken."""
    try:
        text = open(summary).read()
    except OSError:
        return None
    blk = text.split("```json", 1)[-1].split("```", 1)[0] if "```json" in text else ""
    try:
        d = json.loads(blk)
    except ValueError:
        return None
    if d.get("source_hash") != source_hash(sources):
        return None
    return d


def train_probe(heads: int, steps: int = 50, batch: int = 65536):
    """The short program the training-step kernel traces profile: the 5 x 128
    tanh map with `heads` heads, eager lt_map_train_step on one fixed batch
    of 65,536 rays (random targets, half valid), 3 warm-up steps then `steps`
    timed ones, and the same steps as one recorded run (fit.TrainGraph)."""
    import torch
    import paper_2605_04017_amd as lt
    import synth
    dev = torch.device("cuda")
    rays = {k: torch.from_numpy(v).to(dev) for k, v in synth.config_rays(2, batch).items()}
    gen = torch.Generator(device=dev)
    gen.manual_seed(17)
    t = {"valid": (torch.rand((heads, batch), device=dev, generator=gen) > 0.5).to(torch.uint8)}
    for k in ("x", "y", "dx", "dy", "throughput"):
        t[k] = torch.randn((heads, batch), device=dev, generator=gen)
    m = lt.lt_map_create(MAP_WIDTH, MAP_DEPTH, heads, lt.LT_ACT_TANH)
    lt.lt_map_set_params(m, torch.from_numpy(F.init_params(MAP_WIDTH, MAP_DEPTH, heads, 3)).to(dev))
    ws = lt.workspace(m, batch)
    loss = torch.zeros(3, dtype=torch.float32, device=dev)
    for k in range(3):
        lt.lt_map_train_step(m, rays, t, {"lr": 1e-4, "step": k + 1}, ws, loss)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for k in range(steps):
        lt.lt_map_train_step(m, rays, t, {"lr": 1e-4, "step": k + 4}, ws, loss)
    e1.record(stream)
    torch.cuda.synchronize()
    eager = e0.elapsed_time(e1) / steps
    g = F.TrainGraph(m, steps, batch, {}, dev)
    for f, v in g.rays.items():
        v.copy_(rays[f].repeat(steps))
    for f, v in g.targets.items():
        v.copy_(t[f].unsqueeze(0).expand(steps, heads, batch))
    torch.cuda.synchronize()
    e0.record(stream)
    g.run([1e-4] * steps, steps + 4)
    e1.record(stream)
    torch.cuda.synchronize()
    replay = e0.elapsed_time(e1) / steps
    print(json.dumps({"probe": "train", "heads": heads, "batch": batch, "steps": steps,
                      "eager_step_ms": eager, "graph_step_ms": replay}), flush=True)


def traffic_probe(args):
    """Short program for the counter runs: one plain copy of COPY_PROBE_BYTES
    (a negate kernel: reads and writes that many bytes), then three launches
    of the kernel under study.  f32 / bf16 / fp8: the one-head map on the
    4,194,304-ray transmit-only workload (random weights: no data-dependent
    control flow).  trace: three launches of each tracer variant on that
    workload's transmit path.  all_f32 / all_bf16 / all_fp8: the compacted
    56-head map of the headline (16,777,216 rays), fitted exactly as the
    benchmark fits it, so that its valid fraction and output bytes are the
    benchmark's."""
    import torch
    import paper_2605_04017_amd as lt
    import synth
    kind = args.traffic_probe
    dev = torch.device("cuda:0")
    src = torch.ones(COPY_PROBE_BYTES // 4, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    if kind.startswith("all_"):
        n = args.rays_all
        lens = synth.config_lens(3)
        rays = {k: torch.from_numpy(v).to(dev) for k, v in synth.config_rays(3, n).items()}
        h = lt.lt_lens_create(lens.surfaces, lens.glasses)
        paths = all_paths_paths(lens)
        m, _, _, _ = fit_multi_head(lt, synth, lens, h, paths, dev, args.fit_steps)
        dt = {"all_f32": lt.LT_F32, "all_bf16": lt.LT_BF16, "all_fp8": lt.LT_FP8}[kind]
        probe = lt.lt_map_eval_compact(m, lt.LT_F32, rays, capacity=n // 4, with_bits=False)
        cap = int(probe["count"].max()) * 9 // 8 + 1024
        del probe
        torch.cuda.empty_cache()
        cmp = lt.lt_map_eval_compact(m, dt, rays, capacity=cap)
        for _ in range(3):
            lt.lt_map_eval_compact(m, dt, rays, capacity=cap, out=cmp, n=n)
        torch.cuda.synchronize()
        counts = cmp["count"].cpu().tolist()
        print(json.dumps({"probe": "traffic", "kernel": "map compacted, 56 heads", "dtype": kind[4:],
                          "copy_bytes": COPY_PROBE_BYTES, "rays": n, "heads": len(paths),
                          "valid_ray_paths": int(sum(counts)),
                          "algorithmic_bytes": map_compact_bytes(n, len(paths), counts),
                          "source_hash": source_hash(MAP_F32_SOURCES + MAP_BF16_SOURCES)}), flush=True)
        return
    n = args.rays
    rays = {k: torch.from_numpy(v).to(dev) for k, v in synth.config_rays(2, n).items()}
    if kind == "trace":
        h = lt.lt_lens_create(synth.config_lens(2).surfaces, synth.config_lens(2).glasses)
        ex = lt.empty_exit(n, dev)
        for flags in (0, lt.LT_TRACE_PLAIN_FP32, lt.LT_TRACE_FP64):
            for _ in range(3):
                lt.lt_trace_ex(h, (0, 0, 0), rays, ex, n, flags)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "traffic", "kernel": "trace", "copy_bytes": COPY_PROBE_BYTES,
                          "rays": n}), flush=True)
        return
    m = lt.lt_map_create(MAP_WIDTH, MAP_DEPTH, 1, lt.LT_ACT_TANH)
    lt.lt_map_set_params(m, torch.from_numpy(F.init_params(MAP_WIDTH, MAP_DEPTH, 1, 5)).to(dev))
    out = lt.empty_map_out(1, n, dev)
    torch.cuda.synchronize()
    dt = {"f32": lt.LT_F32, "bf16": lt.LT_BF16, "fp8": lt.LT_FP8}[kind]
    for _ in range(3):
        lt.lt_map_eval(m, dt, rays, out, n)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "traffic", "dtype": kind, "copy_bytes": COPY_PROBE_BYTES,
                      "rays": n, "source_hash": source_hash(MAP_F32_SOURCES)}), flush=True)


def transmit_only(lt, synth, dev, args):
    """The 4,194,304-ray transmit-only case: FP32 tracer variants against the
    one-head 5 x 128 map in each precision, map errors, the canonical input."""
    import numpy as np
    import torch
    lens = synth.config_lens(2)
    rays_np = synth.config_rays(2, args.rays)
    n = args.rays
    rays = {k: torch.from_numpy(v).to(dev) for k, v in rays_np.items()}
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    out = lt.empty_exit(n, dev)
    stream = torch.cuda.current_stream()
    t_fit = time.perf_counter()
    m, fitted, fit_loss = fit_map(lt, synth, lens, dev, args.fit_steps)
    t_fit = time.perf_counter() - t_fit
    mout = lt.empty_map_out(1, n, dev)
    reps = 10
    t_trace = time_kernel(lambda: lt.lt_trace(h, (0, 0, 0), rays, out, n, stream), stream, reps)
    t_map = time_kernel(lambda: lt.lt_map_eval(m, lt.LT_F32, rays, mout, n, stream), stream, reps)
    t_bf16 = time_kernel(lambda: lt.lt_map_eval(m, lt.LT_BF16, rays, mout, n, stream), stream, reps)
    t_fp8 = time_kernel(lambda: lt.lt_map_eval(m, lt.LT_FP8, rays, mout, n, stream), stream, reps)
    fast = lt.empty_exit(n, dev)
    t_fast = time_kernel(lambda: lt.lt_trace_ex(h, (0, 0, 0), rays, fast, n, lt.LT_TRACE_PLAIN_FP32,
                                                stream), stream, reps)
    t_f64 = time_kernel(lambda: lt.lt_trace_ex(h, (0, 0, 0), rays, fast, n, lt.LT_TRACE_FP64,
                                               stream), stream, reps)
    errors = {name: map_error(lt, h, m, dt, rays)
              for name, dt in (("f32", lt.LT_F32), ("bf16", lt.LT_BF16), ("fp8", lt.LT_FP8))}
    mc, _, fit_loss_c = fit_map(lt, synth, lens, dev, args.fit_steps, canonical=True)
    errors["f32_canonical_input"] = map_error(lt, h, mc, lt.LT_F32, rays)
    errors["f32_canonical_input"]["fit_final_loss"] = fit_loss_c
    t_map_c = time_kernel(lambda: lt.lt_map_eval(mc, lt.LT_F32, rays, mout, n, stream), stream, 3)
    del mc
    fpr = map_flops_per_ray()
    tfl = trace_flops_per_ray(lens)
    tr = measured_traffic(TRAFFIC_SUMMARY, MAP_F32_SOURCES)
    traffic = None
    if tr is not None and tr.get("rays") == n:
        traffic = tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"]
    res = {
        "workload": "11-surface lens + stop, 4,194,304 sensor-side rays, transmit path; map 5 x 128 tanh, "
                    "1 head (mask logit + x, y, dx, dy, throughput)",
        "rays": n,
        "map_mrays_s": {"f32": n / t_map / 1e6, "bf16": n / t_bf16 / 1e6, "fp8": n / t_fp8 / 1e6},
        "trace_mrays_s": {"float_pair": n / t_trace / 1e6, "fp64_option": n / t_f64 / 1e6,
                          "plain_fp32_outside_tolerance": n / t_fast / 1e6},
        "map_over_trace": {k: {"float_pair": t_trace / t, "fp64_option": t_f64 / t}
                           for k, t in (("f32", t_map), ("bf16", t_bf16), ("fp8", t_fp8))},
        "kernel_ms": {"trace": t_trace * 1e3, "trace_plain_fp32": t_fast * 1e3,
                      "trace_fp64_option": t_f64 * 1e3,
                      "map_f32": t_map * 1e3, "map_bf16": t_bf16 * 1e3, "map_fp8": t_fp8 * 1e3,
                      "map_f32_canonical_input": t_map_c * 1e3},
        "map_error_vs_gpu_tracer": errors,
        "fit": {"steps": args.fit_steps, "batch": 65536, "final_loss": fit_loss, "seconds": t_fit},
        "roofline": {
            "map_f32": {"bound": "mfma", "achieved": fpr * n / t_map / 1e12, "peak": MI355X_FP32_MFMA_TFLOPS,
                        "unit": "TFLOP/s", "frac": fpr * n / t_map / 1e12 / MI355X_FP32_MFMA_TFLOPS,
                        "traffic": traffic, "kernel": "map_eval_f32_kernel<128, tanh>",
                        "flops_per_ray": fpr, "algorithmic_bytes": 53 * n, "traffic_detail": tr},
            "map_bf16": {"bound": "mfma", "achieved": fpr * n / t_bf16 / 1e12,
                         "peak": MI355X_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                         "frac": fpr * n / t_bf16 / 1e12 / MI355X_BF16_MFMA_TFLOPS},
            "map_fp8": {"bound": "mfma", "achieved": fpr * n / t_fp8 / 1e12,
                        "peak": MI355X_FP8_MFMA_TFLOPS, "unit": "TFLOP/s",
                        "frac": fpr * n / t_fp8 / 1e12 / MI355X_FP8_MFMA_TFLOPS},
            "trace": {"bound": "alu", "achieved": tfl * n / t_trace / 1e12, "peak": MI355X_FP32_VECTOR_TFLOPS,
                      "unit": "TFLOP/s", "frac": tfl * n / t_trace / 1e12 / MI355X_FP32_VECTOR_TFLOPS,
                      "flops_per_ray": tfl},
            "trace_fp64_option": {"bound": "alu", "achieved": tfl * n / t_f64 / 1e12,
                                  "peak": MI355X_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                                  "frac": tfl * n / t_f64 / 1e12 / MI355X_FP64_VECTOR_TFLOPS}},
    }
    del rays, out, fast, mout
    torch.cuda.empty_cache()
    return res, lens


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fit-steps", type=int, default=3000)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-transmit-only", action="store_true")
    ap.add_argument("--no-train-epoch", action="store_true")
    ap.add_argument("--no-paper-pair", action="store_true")
    ap.add_argument("--no-paper-recipe", action="store_true")
    ap.add_argument("--paper-recipe-valid", type=int, default=81_000_000,
                    help="valid samples of the paper-recipe fit (the paper's count per path)")
    ap.add_argument("--no-flare", action="store_true")
    ap.add_argument("--no-sampler", action="store_true")
    ap.add_argument("--rays", type=int, default=N_RAYS, help="rays of the transmit-only case")
    ap.add_argument("--rays-all", type=int, default=N_RAYS_ALL_PATHS, help="rays of the 56-path headline")
    ap.add_argument("--traffic-probe", nargs="?", const="f32",
                    choices=("f32", "bf16", "fp8", "trace", "all_f32", "all_bf16", "all_fp8"),
                    help="only run the short program the counter runs profile")
    ap.add_argument("--train-probe", type=int, default=0, metavar="HEADS",
                    help="only time the training step of the 5 x 128 map with this many heads")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: every box in this setup has one MI355X; "
              "multi-GPU sharding is described in DESIGN.md, not run.", file=sys.stderr)
        sys.exit(2)
    if args.traffic_probe:
        traffic_probe(args)
        return
    if args.train_probe:
        train_probe(args.train_probe)
        return

    import torch

    import paper_2605_04017_amd as lt
    import synth

    dev = torch.device("cuda:0")
    A = all_paths(lt, synth, dev, args)
    flat, norms, rays_all_np, lens3, paths = A.pop("_cpu")
    t_trace, t_map, wall = A.pop("_t")
    n, P = args.rays_all, len(paths)
    rl = A["roofline_by_dtype"]["f32"]
    tr = measured_traffic(TRAFFIC_ALL_SUMMARY, MAP_F32_SOURCES + MAP_BF16_SOURCES)
    traffic = None
    if tr is not None and tr.get("rays") == n and tr.get("dtype") == "f32":
        traffic = tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"]
    res = {
        "metric": "Mrays/s map vs GPU brute-force trace at stated exit-ray error; p99 latency",
        "value": P * n / t_map / 1e6,
        "unit": "Mray-paths/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "double-Gauss-style 11-surface lens + stop, 16,777,216 sensor-side rays, "
                               "all 56 paths with at most two reflections (transmit + 55 ghosts); "
                               "step = FP32 brute-force trace of every path (compacted output) + "
                               "FP32 map, one 5 x 128 tanh trunk with 56 heads (compacted output)",
                   "rays": n, "paths": P,
                   "map": "6-D canonical input, 5 x 128 tanh, 56 heads (mask logit + x, y, dx, dy, "
                          f"throughput each), fitted for {args.fit_steps} steps of 65,536 GPU-traced rays"},
        "value_note": "map ray-path evaluations per second (rays x paths), FP32 map; map_over_trace compares "
                      "with each tracer variant that holds 1e-5 mm / 1e-6 rad against the FP64 oracle; the "
                      "BF16 and FP8 maps of the same workload: all_paths_16M (map_over_trace, "
                      "map_error_vs_gpu_tracer and roofline_by_dtype per dtype)",
        "map_over_trace": A["map_over_trace"]["f32"],
        "roofline": {"bound": "mfma", "achieved": rl["achieved"], "peak": rl["peak"], "unit": "TFLOP/s",
                     "frac": rl["frac"], "traffic": traffic,
                     "kernel": "map_eval_f32_kernel<128, tanh, compacted>",
                     "flops_per_ray": rl["flops_per_ray"], "algorithmic_bytes": rl["algorithmic_bytes"],
                     "hbm_achieved_gbs": rl["hbm_gbs"], "hbm_peak_gbs": MI355X_HBM_GBS,
                     "hbm_frac": rl["hbm_frac"], "traffic_detail": tr},
        "roofline_other": {"map_bf16_compact": A["roofline_by_dtype"]["bf16"],
                           "map_fp8_compact": A["roofline_by_dtype"]["fp8"]},
        "all_paths_16M": A,
        "paper_context": {
            "reported": "rendering about 12-15x faster with the maps than with the ray-traced lens "
                        "(depth-of-field path tracing in LuisaRender, per-path 32-wide tanh MLPs)",
            "hardware_and_precision": "not stated in the paper",
            "comparable_here": "map_over_trace (all 56 paths, one trunk with 56 heads) and "
                               "flare_forward frame_speedup_map_over_trace"},
    }
    print("# headline done", file=sys.stderr, flush=True)
    lens2 = None
    if not args.no_transmit_only:
        res["transmit_only_4M"], lens2 = transmit_only(lt, synth, dev, args)
        print("# transmit-only case done", file=sys.stderr, flush=True)
    if not args.no_paper_pair:
        lens2 = lens2 or synth.config_lens(2)
        rays2 = {k: torch.from_numpy(v).to(dev) for k, v in synth.config_rays(2, args.rays).items()}
        res["paper_pair_2x32_5x32"] = paper_pair(lt, synth, lens2, dev, args.fit_steps, rays2)
        del rays2
        print("# paper-size pair done", file=sys.stderr, flush=True)
    if not args.no_paper_recipe:
        res["paper_recipe_ghost"] = paper_recipe(lt, synth, dev, n_valid=args.paper_recipe_valid)
        print("# paper recipe done", file=sys.stderr, flush=True)
    if not args.no_train_epoch:
        res["train_epoch_67M"] = train_epoch(lt, synth, dev)
        print("# training epoch done", file=sys.stderr, flush=True)
    if not args.no_flare:
        res["flare_forward"] = flare(lt, synth, dev)
        print("# flare frame done", file=sys.stderr, flush=True)
    if not args.no_sampler:
        res["sampler_yield_ghost"] = sampler_yield(lt, synth, dev)
        print("# sampler yield done", file=sys.stderr, flush=True)
    if not args.no_serving:
        res["serving"] = serving(lt, synth, dev)
        print("# serving done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_map(flat, norms, rays_all_np, heads=P, canonical=True)
        res["cpu_baseline_trace"] = cpu_baseline_trace(lens3, rays_all_np, paths)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
