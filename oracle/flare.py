"""Sensor image of forward light tracing (Sec. 3, the flare sum over valid
paths; the splat step of the rendering pipeline).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

A ray that leaves a path on the sensor plane at (x, y) with unit direction
w_out and transported intensity I adds I * G to the pixel it lands in, where
h is a box pixel filter and G = dot(w_out, n_cmos) = dz for the sensor
normal n_cmos = +z.  The image of a light source sums this over every valid
path and every sampled ray.

The pixel a ray lands in is an integer decided by floating point, so it is
taken in the precision the library defines it in: FP32 with one rounding
per operation, ix = floor((x - x0) * sx) with x0 = -width/2 and
sx = nx / width rounded to FP32 (likewise y).  The weights are summed in
FP64.
"""
from __future__ import annotations

from typing import Dict, Iterable, Optional, Tuple

import numpy as np

Sensor = Tuple[float, float, int, int]   # width_mm, height_mm, nx, ny


def pixel_of(x: np.ndarray, y: np.ndarray, sensor: Sensor):
    """(inside, ix, iy): the pixel of each exit point, FP32 decision."""
    f32 = np.float32
    w, h, nx, ny = sensor
    x0, y0 = f32(-0.5) * f32(w), f32(-0.5) * f32(h)
    sx, sy = f32(nx) / f32(w), f32(ny) / f32(h)
    with np.errstate(invalid="ignore"):
        u = (np.asarray(x, f32) - x0) * sx
        v = (np.asarray(y, f32) - y0) * sy
        inside = (u >= 0) & (u < f32(nx)) & (v >= 0) & (v < f32(ny))
    ix = np.where(inside, np.floor(np.where(inside, u, 0)), -1).astype(np.int64)
    iy = np.where(inside, np.floor(np.where(inside, v, 0)), -1).astype(np.int64)
    return inside, ix, iy


def splat(x, y, dz, throughput, sensor: Sensor, mask=None, scale: float = 1.0,
          n_per_image: Optional[int] = None) -> np.ndarray:
    """Images [n_images, ny, nx] (float64): ray r adds
    scale * throughput[r] * dz[r] to image r // n_per_image at its pixel."""
    x = np.asarray(x)
    n = x.shape[0]
    n_per_image = n if n_per_image is None else int(n_per_image)
    n_img = max(1, -(-n // n_per_image))
    _, _, nx, ny = sensor
    img = np.zeros((n_img, ny, nx))
    inside, ix, iy = pixel_of(x, y, sensor)
    if mask is not None:
        inside &= np.asarray(mask) != 0
    r = np.flatnonzero(inside)
    wgt = scale * np.asarray(throughput, np.float64)[r] * np.asarray(dz, np.float64)[r]
    np.add.at(img, (r // n_per_image, iy[r], ix[r]), wgt)
    return img


def render_forward(lens, rays: Dict[str, np.ndarray], paths: Iterable, sensor: Sensor,
                   scale: float = 1.0) -> Dict[tuple, np.ndarray]:
    """Per-path sensor images of forward rays traced by the FP64 oracle
    (color[path] of the rendering pipeline); sum them for the final image."""
    import oracle
    out = {}
    for p in paths:
        t = oracle.trace(lens, rays, tuple(p), forward=True)
        out[tuple(p)] = splat(t["x"], t["y"], t["dz"], t["throughput"], sensor,
                              mask=t["mask"], scale=scale)[0]
    return out
