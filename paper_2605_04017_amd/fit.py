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
