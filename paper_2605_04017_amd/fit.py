"""Host-side set-up for fitting maps with the library: seeded initial
parameters in the library's flat layout and normalisation statistics of
inputs and traced targets.  For canonical-input maps the statistics are taken
in the symmetry-reduced frame (Sec. 4.1, geometric simplification), which the
library computes on the device (lt_canonical_frame, the map kernels' own
transform).  None of this runs per ray on the hot path; the training step
itself is lt_map_train_step."""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

N_OUT = 6   # rows per head in the output layer: logit, x, y, dx, dy, throughput


def layer_shapes(width: int, depth: int, n_heads: int) -> List[Tuple[int, int]]:
    """(outputs, inputs) of every layer: 6-D input, depth layers of `width`,
    N_OUT rows per head."""
    return [(width, 6)] + [(width, width)] * (depth - 1) + [(N_OUT * n_heads, width)]


def init_params(width: int, depth: int, n_heads: int, seed: int) -> np.ndarray:
    """Glorot-uniform weights and zero biases as one float32 vector in the
    order lt_map_set_params takes (per layer: weights row-major with the output
    index first, then biases)."""
    rng = np.random.Generator(np.random.Philox(seed))
    parts = []
    for n_out, n_in in layer_shapes(width, depth, n_heads):
        lim = np.sqrt(6.0 / (n_out + n_in))
        parts.append(rng.uniform(-lim, lim, n_out * n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32)


def norm_stats(a: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Column means and standard deviations (1 where a column is constant)."""
    mu, sd = a.mean(0), a.std(0)
    sd = np.where(sd > 0, sd, 1.0)
    return mu, sd


def _canonical(rays: Dict[str, np.ndarray], reg: np.ndarray = None):
    """Rays (and optionally exit rows reg[:, :4] of the same rays) in the
    symmetry-reduced frame, computed on the device by lt_canonical_frame."""
    import torch
    from . import lt_canonical_frame
    dev = torch.device("cuda")
    r = {k: torch.from_numpy(np.ascontiguousarray(rays[k], np.float32)).to(dev)
         for k in ("x", "y", "dx", "dy", "dz", "lambda_nm")}
    ex = None
    if reg is not None:
        ex = {k: torch.from_numpy(np.ascontiguousarray(reg[:, i], np.float32)).to(dev)
              for i, k in enumerate(("x", "y", "dx", "dy"))}
    out = lt_canonical_frame(r, ex, 1, want_rays=reg is None)
    torch.cuda.synchronize()
    if reg is None:
        return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}
    o = np.array(reg, np.float64, copy=True)
    for i, k in enumerate(("x", "y", "dx", "dy")):
        o[:, i] = ex[k].cpu().numpy()
    return o


def map_norms(rays: Dict[str, np.ndarray], targets: List[Tuple[np.ndarray, np.ndarray]],
              canonical: bool = False):
    """(in_shift, in_scale, out_shift [P, 5], out_scale [P, 5]) for a map:
    input statistics over `rays`, and per head the statistics of the traced
    exit (x, y, dx, dy, throughput) over its valid rays.  `targets` holds per
    head (valid mask, [n_valid, 5] exit values of the valid rays); with
    `canonical` both are taken in
    the symmetry-reduced frame."""
    src = _canonical(rays) if canonical else rays
    x = np.stack([np.asarray(src[k], np.float64) for k in ("x", "y", "dx", "dy", "dz", "lambda_nm")], 1)
    in_shift, in_sd = norm_stats(x)
    P = len(targets)
    out_shift, out_scale = np.zeros((P, 5)), np.ones((P, 5))
    for k, (ok, reg) in enumerate(targets):
        ok = np.asarray(ok, bool)
        if ok.sum() < 2:
            continue
        reg = np.asarray(reg, np.float64)
        if canonical:
            sub = {f: np.asarray(rays[f])[ok] for f in ("x", "y", "dx", "dy", "dz", "lambda_nm")}
            reg = _canonical(sub, reg)
        out_shift[k], out_scale[k] = norm_stats(reg)
    return in_shift, 1.0 / in_sd, out_shift, out_scale


# ------------------------------------------------- the paper's training recipe

REG_FIELDS = ("x", "y", "dx", "dy", "throughput")


def paper_lr(step: int, lr0: float = 1e-4, factor: float = 0.95, every: int = 10000) -> float:
    """Sec. 5.1 "MLP Training": the learning rate starts at 1e-4 and decays
    exponentially by 0.95 every 10,000 batches (read as the continuous decay
    lr0 * factor^(step / every), step counted from 0)."""
    return lr0 * factor ** (step / every)


def sampler_dataset(lens, path, n_valid: int, seed: int, n_chains: int = 1 << 20, burn_in: int = 256,
                    thin: int = 8, lambda_mode=None, stream=None) -> Dict:
    """Training data of one path as Sec. 5.1 "Data Collection" describes it,
    drawn and labelled on the device:
    - regressor set: n_valid rays uniform over the path's valid region, from
      Markov chains with a binary visibility target (lt_mcmc_run, one output
      per chain every `thin` steps after `burn_in` steps), wavelengths
      importance-sampled by the CIE matching functions, with their traced
      exit rays (the chains trace every state);
    - classifier set: those valid rays plus as many invalid ones from uniform
      sampling (lt_rays_generate, CIE wavelengths, traced along the path), a
      balanced set.
    Returns {"reg_rays", "reg_exit", "cls_rays", "cls_valid", "chain_steps",
    "uniform_rays"} (device tensors; cls_* shuffled)."""
    import torch
    from . import (LT_LAMBDA_CIE, RAY_FIELDS, lt_mcmc_init, lt_mcmc_run, lt_rays_generate, lt_trace,
                   mcmc_state)
    lam = LT_LAMBDA_CIE if lambda_mode is None else lambda_mode
    dev = torch.device("cuda")
    st = lt_mcmc_init(mcmc_state(n_chains, dev), 0.05, stream=stream)
    rays_b = {k: torch.empty((thin, n_chains), dtype=torch.float32, device=dev) for k in RAY_FIELDS}
    ex_b = None
    first = 0
    for _ in range(max(0, burn_in // thin)):
        rays_b, ex_b, _ = lt_mcmc_run(lens, path, st, thin, seed, first, rays_out=rays_b, exit_out=ex_b,
                                      lambda_mode=lam, stream=stream)
        first += thin
    reg_r = {k: [] for k in RAY_FIELDS}
    reg_e = {k: [] for k in REG_FIELDS}
    have = 0
    while have < n_valid:
        rays_b, ex_b, _ = lt_mcmc_run(lens, path, st, thin, seed, first, rays_out=rays_b, exit_out=ex_b,
                                      lambda_mode=lam, stream=stream)
        first += thin
        ok = ex_b["mask"][thin - 1].bool()
        for k in RAY_FIELDS:
            reg_r[k].append(rays_b[k][thin - 1][ok])
        for k in REG_FIELDS:
            reg_e[k].append(ex_b[k][thin - 1][ok])
        have += int(ok.sum())
    reg_rays = {k: torch.cat(v)[:n_valid].contiguous() for k, v in reg_r.items()}
    reg_exit = {k: torch.cat(v)[:n_valid].contiguous() for k, v in reg_e.items()}
    # invalid rays of the uniform distribution
    inv = {k: [] for k in RAY_FIELDS}
    have, n_uniform, chunk, k0 = 0, 0, max(n_valid, 1 << 20), 0
    while have < n_valid:
        u = lt_rays_generate(lens, chunk, seed + 1, first=k0, lambda_mode=lam, stream=stream)
        k0 += chunk
        n_uniform += chunk
        bad = lt_trace(lens, path, u, stream=stream)["mask"] == 0
        for k in RAY_FIELDS:
            inv[k].append(u[k][bad])
        have += int(bad.sum())
    inv_rays = {k: torch.cat(v)[:n_valid] for k, v in inv.items()}
    g = torch.Generator(device=dev)
    g.manual_seed(seed + 2)
    perm = torch.randperm(2 * n_valid, device=dev, generator=g)
    cls_rays = {k: torch.cat([reg_rays[k], inv_rays[k]])[perm].contiguous() for k in RAY_FIELDS}
    cls_valid = torch.cat([torch.ones(n_valid, dtype=torch.uint8, device=dev),
                           torch.zeros(n_valid, dtype=torch.uint8, device=dev)])[perm].contiguous()
    return {"reg_rays": reg_rays, "reg_exit": reg_exit, "cls_rays": cls_rays, "cls_valid": cls_valid,
            "chain_steps": first * n_chains, "uniform_rays": n_uniform}


def fit_epochs(m, rays: Dict, targets: Dict, epochs: int, batch: int, cfg: Dict, seed: int,
               lr=paper_lr, stream=None, graph_steps: int = 0):
    """Adam over `epochs` shuffled passes of a fixed dataset (rays: dict of
    [n] device tensors; targets: dict of [1, n] tensors as lt_map_train_step
    takes them), `batch` rays per step, the learning rate lr(step) from step 0
    (the paper's schedule by default).  cfg: the loss weights.  With
    graph_steps > 0 the steps run in recorded runs of that many steps
    (TrainGraph; each run's shuffled batches gathered into its buffers), the
    last steps of an epoch that do not fill a run eagerly; the result is the
    same as the eager loop's.  Returns (steps, last loss tensor)."""
    import torch
    from . import lt_map_train_step, workspace
    n = int(rays["x"].numel())
    per_epoch = n // batch
    dev = rays["x"].device
    ws = workspace(m, batch)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    K = min(int(graph_steps), per_epoch)
    G = TrainGraph(m, K, batch, cfg, dev) if K > 0 else None
    P = m.n_heads
    step, loss = 0, None
    for _ in range(epochs):
        perm = torch.randperm(n, device=dev, generator=g)
        b = 0
        if G is not None:
            while b + K <= per_epoch:
                idx = perm[b * batch:(b + K) * batch]
                for f, v in G.rays.items():
                    torch.index_select(rays[f], 0, idx, out=v)
                for f, v in G.targets.items():
                    v.copy_(targets[f].index_select(1, idx).reshape(P, K, batch).permute(1, 0, 2))
                loss = G.run([lr(step + k) for k in range(K)], step + 1)[K - 1]
                step += K
                b += K
            if b == per_epoch:
                continue
        R = {k: v[perm] for k, v in rays.items()}
        T = {k: v[:, perm] for k, v in targets.items()}
        for bb in range(b, per_epoch):
            lo = bb * batch
            rb = {k: v[lo:lo + batch] for k, v in R.items()}
            tb = {k: v[:, lo:lo + batch] for k, v in T.items()}
            c = dict(cfg)
            c["lr"] = lr(step)
            step += 1
            c["step"] = step
            loss = lt_map_train_step(m, rb, tb, c, ws, stream=stream)
    return step, loss


class TrainGraph:
    """A run of `steps` fused training steps (lt_map_train_step: forward,
    loss, backward, reduce + Adam, with the two repacks) recorded once into
    one HIP graph and replayed, so a run costs one graph launch instead of
    eight kernel launches and the wrapper's marshalling per step.

    Step k of a run trains on rays [k * batch, (k + 1) * batch) of the static
    buffers `rays` (dict of [steps * batch] tensors) and on targets[f][k]
    (`targets`: dict of [steps, n_heads, batch] tensors); fill them before
    run(), e.g. with a gather of the next shuffled batches.  Learning rate and
    step count come from a device array of lt_train_sched entries that run()
    writes with one copy, so one recording serves every run.  Replays and
    eager calls on the same map may be mixed: each recorded step repacks the
    parameters before its forward, and run() marks the map updated
    (lt_map_mark_updated) so that the next eager evaluation repacks too.  The
    map must not be trained or have its parameters set by other calls while a
    replay is in flight."""

    def __init__(self, m, steps: int, batch: int, cfg: Dict, device="cuda"):
        import torch
        from . import RAY_FIELDS, TARGET_FIELDS, lt_map_train_step, workspace
        self.m, self.steps, self.batch = m, int(steps), int(batch)
        P = m.n_heads
        self.rays = {k: torch.zeros(steps * batch, dtype=torch.float32, device=device) for k in RAY_FIELDS}
        self.targets = {k: torch.zeros((steps, P, batch), dtype=torch.uint8 if k == "valid" else torch.float32,
                                       device=device) for k in TARGET_FIELDS}
        self.ws = workspace(m, batch, device)
        self.loss = torch.zeros((steps, 3), dtype=torch.float32, device=device)
        self.sched = torch.zeros((steps, 16), dtype=torch.uint8, device=device)
        c = {k: v for k, v in cfg.items() if k not in ("lr", "step")}
        self.graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(self.graph):
            st = torch.cuda.current_stream()
            for k in range(self.steps):
                rb = {f: v[k * batch:(k + 1) * batch] for f, v in self.rays.items()}
                tb = {f: v[k] for f, v in self.targets.items()}
                lt_map_train_step(m, rb, tb, dict(c, sched=self.sched[k]), self.ws, self.loss[k], batch, st)
        torch.cuda.synchronize()

    def run(self, lrs, first_step: int):
        """Replay the recorded steps with learning rates lrs[k] and step
        counts first_step + k (1-based); returns the device losses
        [steps, 3] (total, BCE, L2 per step)."""
        import numpy as np
        import torch
        from . import lt_map_mark_updated
        assert len(lrs) == self.steps
        host = np.zeros(self.steps, dtype=[("lr", "<f4"), ("reserved", "<i4"), ("step", "<i8")])
        host["lr"] = np.asarray(lrs, np.float32)
        host["step"] = first_step + np.arange(self.steps, dtype=np.int64)
        self.sched.copy_(torch.from_numpy(host.view(np.uint8).reshape(self.steps, 16)))
        self.graph.replay()
        lt_map_mark_updated(self.m)
        return self.loss

