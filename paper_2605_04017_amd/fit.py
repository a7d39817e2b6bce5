"""Host-side set-up for fitting maps with the library: seeded initial
parameters in the library's flat layout, normalisation statistics of inputs
and traced targets, and the symmetry-reduced frame those statistics are taken
in for canonical-input maps (Sec. 4.1, geometric simplification).  None of
this runs per ray on the hot path; the training step itself is
lt_map_train_step."""
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


def canonical_rotation(x: np.ndarray, y: np.ndarray, dx: np.ndarray, dy: np.ndarray):
    """Rotation (c, s) taking the sensor point onto the +x half line and the
    mirror flag making the rotated direction's y component non-negative (the
    identity rotation for a point on the axis)."""
    x, y, dx, dy = (np.asarray(v, np.float64) for v in (x, y, dx, dy))
    r = np.hypot(x, y)
    on_axis = r == 0
    rr = np.where(on_axis, 1.0, r)
    c = np.where(on_axis, 1.0, x / rr)
    s = np.where(on_axis, 0.0, y / rr)
    flip = (c * dy - s * dx) < 0
    return c, s, flip


def canonical_inputs(rays: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """Sensor-side rays in their symmetry-reduced frame (float64): r, 0,
    rotated (and mirrored) direction, dz and wavelength unchanged."""
    c, s, flip = canonical_rotation(rays["x"], rays["y"], rays["dx"], rays["dy"])
    x, y, dx, dy = (np.asarray(rays[k], np.float64) for k in ("x", "y", "dx", "dy"))
    m = np.where(flip, -1.0, 1.0)
    return {"x": c * x + s * y, "y": np.zeros_like(x), "dx": c * dx + s * dy,
            "dy": m * (c * dy - s * dx), "dz": np.asarray(rays["dz"], np.float64),
            "lambda_nm": np.asarray(rays["lambda_nm"], np.float64)}


def canonical_outputs(rays: Dict[str, np.ndarray], out: np.ndarray) -> np.ndarray:
    """Exit (x, y, dx, dy, ...) columns of `out` (rows = the given rays) moved
    into each ray's symmetry-reduced frame; further columns unchanged."""
    c, s, flip = canonical_rotation(rays["x"], rays["y"], rays["dx"], rays["dy"])
    m = np.where(flip, -1.0, 1.0)
    o = np.array(out, np.float64, copy=True)
    x, y, dx, dy = o[:, 0].copy(), o[:, 1].copy(), o[:, 2].copy(), o[:, 3].copy()
    o[:, 0], o[:, 1] = c * x + s * y, m * (c * y - s * x)
    o[:, 2], o[:, 3] = c * dx + s * dy, m * (c * dy - s * dx)
    return o


def map_norms(rays: Dict[str, np.ndarray], targets: List[Tuple[np.ndarray, np.ndarray]],
              canonical: bool = False):
    """(in_shift, in_scale, out_shift [P, 5], out_scale [P, 5]) for a map:
    input statistics over `rays`, and per head the statistics of the traced
    exit (x, y, dx, dy, throughput) over its valid rays.  `targets` holds per
    head (valid mask, [n, 5] exit values); with `canonical` both are taken in
    the symmetry-reduced frame."""
    src = canonical_inputs(rays) if canonical else rays
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
            sub = {f: np.asarray(rays[f])[ok] for f in ("x", "y", "dx", "dy")}
            reg = canonical_outputs(sub, reg)
        out_shift[k], out_scale[k] = norm_stats(reg)
    return in_shift, 1.0 / in_sd, out_shift, out_scale
