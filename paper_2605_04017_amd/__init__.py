"""MI355X-native lens transport maps (arXiv 2605.04017): Python binding.

The functions here carry the names of the C ABI in include/lt.h and only
marshal arguments: every per-ray step runs in the HIP kernels of liblt.so.
Device buffers are torch tensors (PyTorch provides memory and streams only).
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence, Tuple

from . import _native as N
from ._native import LtError

RAY_FIELDS = ("x", "y", "dx", "dy", "dz", "lambda_nm")
EXIT_FIELDS = ("mask", "x", "y", "dx", "dy", "dz", "throughput")

LT_TRACE_PLAIN_FP32 = N.LT_TRACE_PLAIN_FP32
LT_TRACE_FORWARD = N.LT_TRACE_FORWARD
LT_TRACE_FP64 = N.LT_TRACE_FP64
LT_LAMBDA_UNIFORM, LT_LAMBDA_CIE = N.LT_LAMBDA_UNIFORM, N.LT_LAMBDA_CIE
LT_F32, LT_BF16, LT_FP8 = N.LT_F32, N.LT_BF16, N.LT_FP8
LT_ACT_TANH, LT_ACT_RELU = N.LT_ACT_TANH, N.LT_ACT_RELU
MAP_FIELDS = ("logit", "mask", "x", "y", "dx", "dy", "dz", "throughput")
LT_ERR_ARG, LT_ERR_STATE = N.LT_ERR_ARG, N.LT_ERR_STATE
LT_STATIC_SCRATCH_BYTES = N.LT_STATIC_SCRATCH_BYTES

__all__ = ["LtError", "Lens", "lt_lens_create", "lt_lens_query", "lt_lens_paraxial", "lt_canonical_frame", "lt_trace", "lt_trace_ex",
           "lt_ghost_index", "lt_ghost_path", "empty_exit", "RAY_FIELDS", "EXIT_FIELDS",
           "LT_TRACE_PLAIN_FP32", "LT_F32", "LT_BF16", "LT_FP8", "LT_ACT_TANH", "LT_ACT_RELU",
           "Map", "lt_map_create", "lt_map_set_params", "lt_map_get_params", "lt_map_set_norm",
           "lt_map_eval", "empty_map_out", "MAP_FIELDS", "lt_map_workspace_bytes", "workspace",
           "lt_map_forward_train", "lt_map_backward", "lt_map_train_step", "lt_map_train_step_static",
           "lt_map_adam_state", "LT_STATIC_SCRATCH_BYTES",
           "TARGET_FIELDS", "lt_path_encode", "lt_path_decode", "lt_trace_compact",
           "lt_map_quantize", "lt_rays_generate", "lt_map_eval_ex", "LT_EVAL_MASK_ONLY",
           "lt_lens_planes", "LT_TRACE_FORWARD", "LT_TRACE_FP64", "lt_rays_generate_forward", "lt_splat",
           "LT_LAMBDA_UNIFORM", "LT_LAMBDA_CIE", "mcmc_state", "lt_mcmc_init", "lt_mcmc_run",
           "LT_EVAL_GATED", "Server", "LT_ERR_ARG", "LT_ERR_STATE", "train_sched", "set_train_sched", "lt_map_mark_updated",
           "lt_mask_index", "lt_map_eval_indexed"]

TARGET_FIELDS = ("valid", "x", "y", "dx", "dy", "throughput")


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev_ptr(t, dtype, n: int, name: str) -> int:
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: tensor must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{name}: has {t.numel()} elements, need {n}")
    return t.data_ptr()


class Lens:
    """Owned lt_lens handle."""

    def __init__(self, handle: int, n_surfaces: int, n_refracting: int, n_ghost: int,
                 front_semi_diameter: float = 0.0):
        self._h = C.c_void_p(handle)
        self.n_surfaces = n_surfaces
        self.n_refracting = n_refracting
        self.n_ghost_paths = n_ghost
        self.front_semi_diameter = front_semi_diameter

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            N.lib().lt_lens_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _surface_rows(surfaces):
    rows = []
    for s in surfaces:
        if hasattr(s, "radius"):
            rows.append((s.radius, s.thickness, s.semi_diameter, s.glass_after, s.is_stop))
        else:
            rows.append(tuple(s))
    return rows


def _glass_rows(glasses):
    rows = []
    for g in glasses:
        if hasattr(g, "kind"):
            rows.append((g.kind, *g.coef))
        else:
            rows.append(tuple(g))
    return rows


def lt_lens_create(surfaces, glasses) -> Lens:
    """Validate and store a prescription.  ``surfaces``: rows (radius,
    thickness, semi_diameter, glass_after, is_stop) or objects with those
    attributes; ``glasses``: rows (kind, c0..c5) or objects with kind/coef."""
    srows = _surface_rows(surfaces)
    grows = _glass_rows(glasses)
    S = (N.lt_surface * max(1, len(srows)))()
    for k, (r, t, sd, ga, st) in enumerate(srows):
        S[k].radius_mm, S[k].thickness_mm, S[k].semi_diameter_mm = float(r), float(t), float(sd)
        S[k].glass_after, S[k].is_stop = int(ga), int(st)
    G = (N.lt_glass * max(1, len(grows)))()
    for k, row in enumerate(grows):
        G[k].kind = int(row[0])
        for m in range(6):
            G[k].coef[m] = float(row[1 + m]) if 1 + m < len(row) else 0.0
    h = C.c_void_p()
    N.check(N.lib().lt_lens_create(S, len(srows), G, len(grows), C.byref(h)))
    ns, nr, ng = C.c_int32(), C.c_int32(), C.c_int32()
    N.check(N.lib().lt_lens_query(h, C.byref(ns), C.byref(nr), C.byref(ng), None, None))
    return Lens(h.value, ns.value, nr.value, ng.value, float(srows[0][2]) if srows else 0.0)


def lt_lens_query(lens: Lens) -> Tuple[int, int, int, float, float]:
    """(surfaces, refracting surfaces, ghost paths, paraxial EFL, back focal
    distance) with the focal lengths in mm at the d line (587.5618 nm)."""
    ns, nr, ng = C.c_int32(), C.c_int32(), C.c_int32()
    efl, bfl = C.c_double(), C.c_double()
    N.check(N.lib().lt_lens_query(lens.handle, C.byref(ns), C.byref(nr), C.byref(ng),
                                  C.byref(efl), C.byref(bfl)))
    return ns.value, nr.value, ng.value, efl.value, bfl.value


def lt_lens_paraxial(lens: Lens, lambda_nm: float) -> Tuple[float, float]:
    """Paraxial (EFL, back focal distance) in mm at ``lambda_nm``."""
    efl, bfl = C.c_double(), C.c_double()
    N.check(N.lib().lt_lens_paraxial(lens.handle, float(lambda_nm), C.byref(efl), C.byref(bfl)))
    return efl.value, bfl.value


def lt_lens_planes(lens: Lens) -> Tuple[float, float]:
    """(z of the forward input plane, z of the sensor plane) in the lens frame."""
    a, b = C.c_double(), C.c_double()
    N.check(N.lib().lt_lens_planes(lens.handle, C.byref(a), C.byref(b)))
    return a.value, b.value


def lt_ghost_index(n_refracting: int, j: int, i: int) -> int:
    return int(N.lib().lt_ghost_index(n_refracting, j, i))


def lt_ghost_path(n_refracting: int, index: int) -> Tuple[int, int, int]:
    p = N.lt_path()
    N.check(N.lib().lt_ghost_path(n_refracting, index, C.byref(p)))
    return (p.kind, p.j, p.i)


def lt_path_encode(n_refracting: int, path) -> int:
    """Binary id of a path: sentinel 1, then one bit per refracting-surface
    interaction in scene-to-sensor order (reflect = 1)."""
    v = C.c_uint64()
    p = _path(path)
    N.check(N.lib().lt_path_encode(n_refracting, C.byref(p), C.byref(v)))
    return int(v.value)


def lt_path_decode(n_refracting: int, path_id: int) -> Tuple[int, int, int]:
    p = N.lt_path()
    N.check(N.lib().lt_path_decode(n_refracting, int(path_id), C.byref(p)))
    return (p.kind, p.j, p.i)


def _path(path) -> N.lt_path:
    if isinstance(path, N.lt_path):
        return path
    k, j, i = (tuple(path) + (0, 0, 0))[:3]
    return N.lt_path(int(k), int(j), int(i))


def _rays_struct(rays: Dict, n: int) -> N.lt_rays:
    torch = _torch()
    r = N.lt_rays()
    for k in RAY_FIELDS:
        setattr(r, k, _dev_ptr(rays[k], torch.float32, n, f"rays[{k}]") if n else None)
    return r


def empty_exit(n: int, device="cuda") -> Dict:
    torch = _torch()
    out = {"mask": torch.empty(n, dtype=torch.uint8, device=device)}
    for k in EXIT_FIELDS[1:]:
        out[k] = torch.empty(n, dtype=torch.float32, device=device)
    return out


def lt_trace(lens: Lens, path, rays: Dict, out: Optional[Dict] = None, n: Optional[int] = None,
             stream=None) -> Dict:
    """Brute-force FP32 trace of ``n`` sensor-side rays along ``path``
    ((0,0,0) = transmit, (1, j, i) = ghost).  ``rays``: dict of float32 CUDA
    tensors; ``out``: dict of exit tensors (allocated if None)."""
    return lt_trace_ex(lens, path, rays, out, n, 0, stream)


def lt_trace_ex(lens: Lens, path, rays: Dict, out: Optional[Dict] = None,
                n: Optional[int] = None, flags: int = 0, stream=None) -> Dict:
    """lt_trace with option flags (LT_TRACE_PLAIN_FP32 = 1, LT_TRACE_FORWARD = 2,
    LT_TRACE_FP64 = 4)."""
    torch = _torch()
    if n is None:
        n = int(rays["x"].numel())
    if out is None:
        out = empty_exit(n, rays["x"].device)
    e = N.lt_exit()
    for k in EXIT_FIELDS:
        dt = torch.uint8 if k == "mask" else torch.float32
        setattr(e, k, _dev_ptr(out[k], dt, n, f"out[{k}]") if n else None)
    p = _path(path)
    N.check(N.lib().lt_trace_ex(lens.handle, C.byref(p), C.byref(_rays_struct(rays, n)),
                                C.byref(e), int(n), int(flags),
                                C.c_void_p(_stream_ptr(stream) if n else 0)))
    return out


def lt_rays_generate(lens: Lens, n: int, seed: int, first: int = 0, half_width: float = 18.0,
                     half_height: float = 12.0, lam_range=(400.0, 700.0), out: Optional[Dict] = None,
                     device="cuda", stream=None, lambda_mode: int = N.LT_LAMBDA_UNIFORM) -> Dict:
    """n sensor-side rays drawn on the device (Philox4x64-10, ray k from
    counter first + k); returns a dict of float32 tensors."""
    torch = _torch()
    if out is None:
        out = {k: torch.empty(n, dtype=torch.float32, device=device) for k in RAY_FIELDS}
    b = N.lt_ray_buffers()
    for k in RAY_FIELDS:
        setattr(b, k, _dev_ptr(out[k], torch.float32, n, f"out[{k}]") if n else None)
    cfg = N.lt_raygen(int(seed) & 0xFFFFFFFFFFFFFFFF, int(first) & 0xFFFFFFFFFFFFFFFF,
                      float(half_width), float(half_height), float(lam_range[0]),
                      float(lam_range[1]), int(lambda_mode))
    N.check(N.lib().lt_rays_generate(lens.handle, C.byref(cfg), C.byref(b), int(n),
                                     C.c_void_p(_stream_ptr(stream) if n else 0)))
    return out


def lt_canonical_frame(rays: Dict, exits: Optional[Dict] = None, n_heads: int = 1,
                       out: Optional[Dict] = None, want_rays: bool = True,
                       n: Optional[int] = None, stream=None) -> Optional[Dict]:
    """Symmetry-reduced frame of a canonical-input map (the map kernels' own
    transform): returns the canonical rays (dict of float32 tensors) unless
    ``want_rays`` is False; ``exits`` (dict with x, y, dx, dy float32 tensors of
    n_heads * n entries, head-major) is moved into each ray's frame in place."""
    torch = _torch()
    if n is None:
        n = int(rays["x"].numel())
    ro = None
    if want_rays:
        if out is None:
            out = {k: torch.empty(n, dtype=torch.float32, device=rays["x"].device)
                   for k in RAY_FIELDS}
        ro = N.lt_ray_buffers()
        for k in RAY_FIELDS:
            setattr(ro, k, _dev_ptr(out[k], torch.float32, n, f"out[{k}]") if n else None)
    ex = None
    if exits is not None:
        ex = N.lt_exit()
        for k in ("x", "y", "dx", "dy"):
            setattr(ex, k, _dev_ptr(exits[k], torch.float32, n_heads * n, f"exits[{k}]") if n else None)
    N.check(N.lib().lt_canonical_frame(C.byref(_rays_struct(rays, n)),
                                       C.byref(ro) if ro is not None else None,
                                       C.byref(ex) if ex is not None else None,
                                       int(n_heads if exits is not None else 0), int(n),
                                       C.c_void_p(_stream_ptr(stream) if n else 0)))
    return out if want_rays else None


def lt_rays_generate_forward(lens: Lens, n: int, seed: int, light=(0.0, 0.0, 1.0),
                             at_infinity: bool = True, aperture: Optional[float] = None,
                             first: int = 0, lam_range=(400.0, 700.0), out: Optional[Dict] = None,
                             device="cuda", stream=None) -> Dict:
    """n scene-side rays from a point light drawn on the device (p_in
    uniform on the aperture disk of the forward input plane).  ``light``: the
    direction of travel (at infinity) or the light's position.  ``aperture``
    defaults to the first surface's semi-diameter."""
    torch = _torch()
    if aperture is None:
        aperture = lens.front_semi_diameter
    if out is None:
        out = {k: torch.empty(n, dtype=torch.float32, device=device) for k in RAY_FIELDS}
    b = N.lt_ray_buffers()
    for k in RAY_FIELDS:
        setattr(b, k, _dev_ptr(out[k], torch.float32, n, f"out[{k}]") if n else None)
    cfg = N.lt_raygen_forward(int(seed) & 0xFFFFFFFFFFFFFFFF, int(first) & 0xFFFFFFFFFFFFFFFF,
                              (C.c_float * 3)(*[float(v) for v in light]), int(bool(at_infinity)),
                              float(aperture), float(lam_range[0]), float(lam_range[1]))
    N.check(N.lib().lt_rays_generate_forward(lens.handle, C.byref(cfg), C.byref(b), int(n),
                                             C.c_void_p(_stream_ptr(stream) if n else 0)))
    return out


def mcmc_state(n_chains: int, device="cuda") -> Dict:
    """Device buffers of n_chains Markov chains (u [5][n], step, n_small,
    visible); call lt_mcmc_init before the first run."""
    torch = _torch()
    return {"u": torch.empty((5, n_chains), dtype=torch.float32, device=device),
            "step": torch.empty(n_chains, dtype=torch.float32, device=device),
            "n_small": torch.empty(n_chains, dtype=torch.int32, device=device),
            "visible": torch.empty(n_chains, dtype=torch.uint8, device=device)}


def _mcmc_struct(state) -> "N.lt_mcmc_state":
    torch = _torch()
    n = int(state["step"].numel())
    s = N.lt_mcmc_state()
    if n:
        s.u = _dev_ptr(state["u"], torch.float32, 5 * n, "state[u]")
        s.step = _dev_ptr(state["step"], torch.float32, n, "state[step]")
        s.n_small = _dev_ptr(state["n_small"], torch.int32, n, "state[n_small]")
        s.visible = _dev_ptr(state["visible"], torch.uint8, n, "state[visible]")
    return s


def lt_mcmc_init(state: Dict, step0: float = 0.05, stream=None):
    n = int(state["step"].numel())
    N.check(N.lib().lt_mcmc_init(C.byref(_mcmc_struct(state)), n, float(step0),
                                 C.c_void_p(_stream_ptr(stream) if n else 0)))
    return state


def lt_mcmc_run(lens: Lens, path, state: Dict, n_steps: int, seed: int, first_step: int = 0,
                p_large: float = 0.1, target_accept: float = 0.234, half_width: float = 18.0,
                half_height: float = 12.0, lam_range=(400.0, 700.0),
                lambda_mode: int = N.LT_LAMBDA_UNIFORM, rays_out: Optional[Dict] = None,
                exit_out: Optional[Dict] = None, counts=None, flags: int = 0, stream=None):
    """Advance the chains by n_steps along ``path``; returns (rays, exits,
    counts): rays / exits are dicts of [n_steps, n_chains] tensors (step-major),
    counts a device uint64[4] (independent proposals, accepted, small steps,
    accepted), accumulated into if given."""
    torch = _torch()
    n = int(state["step"].numel())
    dev = state["step"].device
    m = n * int(n_steps)
    if rays_out is None:
        rays_out = {k: torch.empty((n_steps, n), dtype=torch.float32, device=dev) for k in RAY_FIELDS}
    if exit_out is None:
        exit_out = empty_exit(m, dev)
        exit_out = {k: v.view(n_steps, n) for k, v in exit_out.items()}
    if counts is None:
        counts = torch.zeros(4, dtype=torch.int64, device=dev)
    rb = N.lt_ray_buffers()
    eb = N.lt_exit()
    for k in RAY_FIELDS:
        setattr(rb, k, _dev_ptr(rays_out[k], torch.float32, m, f"rays_out[{k}]") if m else None)
    for k in EXIT_FIELDS:
        dt = torch.uint8 if k == "mask" else torch.float32
        setattr(eb, k, _dev_ptr(exit_out[k], dt, m, f"exit_out[{k}]") if m else None)
    cfg = N.lt_mcmc_cfg(int(seed) & 0xFFFFFFFFFFFFFFFF, int(first_step) & 0xFFFFFFFFFFFFFFFF,
                        float(half_width), float(half_height), float(lam_range[0]),
                        float(lam_range[1]), int(lambda_mode), float(p_large), float(target_accept))
    cp = _dev_ptr(counts, torch.int64, 4, "counts") if n else None
    N.check(N.lib().lt_mcmc_run(lens.handle, C.byref(_path(path)), C.byref(cfg),
                                C.byref(_mcmc_struct(state)), n, int(n_steps), C.byref(rb),
                                C.byref(eb), cp, int(flags),
                                C.c_void_p(_stream_ptr(stream) if n else 0)))
    return rays_out, exit_out, counts


def lt_splat(x, y, dz, throughput, sensor, images=None, mask=None, n: Optional[int] = None,
             n_per_image: Optional[int] = None, scale: float = 1.0, stream=None):
    """Add scale * throughput * dz of every (masked) exit ray to its sensor
    pixel; ``sensor`` = (width_mm, height_mm, nx, ny).  ``images`` (float32,
    [n_images, ny, nx], accumulated into) is allocated zeroed if None."""
    torch = _torch()
    if n is None:
        n = int(x.numel())
    per = max(1, n) if n_per_image is None else int(n_per_image)
    w, h, nx, ny = sensor
    n_img = max(1, -(-n // max(1, per)))
    if images is None:
        images = torch.zeros((n_img, int(ny), int(nx)), dtype=torch.float32, device=x.device)
    s = N.lt_sensor(float(w), float(h), int(nx), int(ny))
    f32 = torch.float32
    ptrs = [_dev_ptr(t, f32, n, nm) if n else None
            for t, nm in ((x, "x"), (y, "y"), (dz, "dz"), (throughput, "throughput"))]
    mp = _dev_ptr(mask, torch.uint8, n, "mask") if (mask is not None and n) else None
    ip = _dev_ptr(images, f32, n_img * int(nx) * int(ny), "images") if n else None
    N.check(N.lib().lt_splat(*ptrs, mp, int(n), int(per), C.byref(s), float(scale), ip,
                             C.c_void_p(_stream_ptr(stream) if n else 0)))
    return images


def lt_trace_compact(lens: Lens, path, rays: Dict, out: Optional[Dict] = None, idx=None,
                     count=None, n: Optional[int] = None, flags: int = 0, stream=None):
    """Trace and keep only valid rays: returns (out, idx, count) where the
    first count[0] entries of out[x .. throughput] are the exit rays of input
    rays idx[:count[0]] (block order unspecified; sort by idx for a canonical
    order)."""
    torch = _torch()
    if n is None:
        n = int(rays["x"].numel())
    dev = rays["x"].device
    if out is None:
        out = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in EXIT_FIELDS[1:]}
    if idx is None:
        idx = torch.empty(n, dtype=torch.int64, device=dev)
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=dev)
    e = N.lt_exit()
    for k in EXIT_FIELDS[1:]:
        setattr(e, k, _dev_ptr(out[k], torch.float32, n, f"out[{k}]") if n else None)
    e.mask = None
    p = _path(path)
    N.check(N.lib().lt_trace_compact(lens.handle, C.byref(p), C.byref(_rays_struct(rays, n)),
                                     C.byref(e), _dev_ptr(idx, torch.int64, n, "idx") if n else None,
                                     _dev_ptr(count, torch.int64, 1, "count"), int(n), int(flags),
                                     C.c_void_p(_stream_ptr(stream))))
    return out, idx, count


# ------------------------------------------------------------------- map --

class Map:
    """Owned lt_map handle."""

    def __init__(self, handle: int, width: int, depth: int, n_heads: int, activation: int):
        self._h = C.c_void_p(handle)
        self.width, self.depth, self.n_heads, self.activation = width, depth, n_heads, activation
        self.n_params = int(N.lib().lt_map_num_params(self._h))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            N.lib().lt_map_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lt_map_create(width: int = 128, depth: int = 5, n_heads: int = 1,
                  activation: int = N.LT_ACT_TANH, canonical: bool = False,
                  forward: bool = False) -> Map:
    """``canonical``: symmetry-reduced input frame (rotation + mirror about
    the optical axis); ``forward``: a forward-light-tracing map (exit dz > 0).
    See lt_map_desc in include/lt.h."""
    d = N.lt_map_desc(6, int(width), int(depth), int(n_heads), int(activation), int(bool(canonical)),
                      int(bool(forward)))
    h = C.c_void_p()
    N.check(N.lib().lt_map_create(C.byref(d), C.byref(h)))
    m = Map(h.value, width, depth, n_heads, activation)
    m.canonical = bool(canonical)
    m.forward = bool(forward)
    return m


def lt_map_set_params(m: Map, params, stream=None):
    """``params``: float32 CUDA tensor with m.n_params entries (FP32 master)."""
    torch = _torch()
    ptr = _dev_ptr(params, torch.float32, m.n_params, "params")
    N.check(N.lib().lt_map_set_params(m.handle, C.c_void_p(ptr), m.n_params,
                                      C.c_void_p(_stream_ptr(stream))))


def lt_map_get_params(m: Map, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty(m.n_params, dtype=torch.float32, device="cuda")
    ptr = _dev_ptr(out, torch.float32, m.n_params, "out")
    N.check(N.lib().lt_map_get_params(m.handle, C.c_void_p(ptr), m.n_params,
                                      C.c_void_p(_stream_ptr(stream))))
    return out


def lt_map_set_norm(m: Map, in_shift, in_scale, out_shift, out_scale):
    import numpy as np

    def arr(a, k):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1))
        if a.size != k:
            raise ValueError(f"expected {k} values, got {a.size}")
        return a
    P = m.n_heads
    a = [arr(in_shift, 6), arr(in_scale, 6), arr(out_shift, 5 * P), arr(out_scale, 5 * P)]
    fp = C.POINTER(C.c_float)
    N.check(N.lib().lt_map_set_norm(m.handle, *[x.ctypes.data_as(fp) for x in a]))


def empty_map_out(n_heads: int, n: int, device="cuda") -> Dict:
    torch = _torch()
    out = {}
    for k in MAP_FIELDS:
        out[k] = torch.empty((n_heads, n), dtype=torch.uint8 if k == "mask" else torch.float32,
                             device=device)
    return out


def lt_map_quantize(m: Map, dtype: int, stream=None) -> None:
    """Build the packed weights lt_map_eval uses for ``dtype`` now."""
    N.check(N.lib().lt_map_quantize(m.handle, int(dtype), C.c_void_p(_stream_ptr(stream))))


def lt_map_eval(m: Map, dtype: int, rays: Dict, out: Optional[Dict] = None,
                n: Optional[int] = None, stream=None) -> Dict:
    """Evaluate the map for ``n`` rays; outputs are (n_heads, n) tensors."""
    return lt_map_eval_ex(m, dtype, rays, out, n, 0, None, stream)


# --------------------------------------------------------------- serving --

class Server:
    """Owned lt_server handle: the native continuous-batching request loop
    (lt_server_* in include/lt.h).  Requests keep their tensors alive here
    until they are reported done."""

    def __init__(self, n_streams: int = 4, chunk: int = 262144, mem_budget: int = 4 << 30,
                 bytes_per_ray: int = 64):
        cfg = N.lt_server_cfg(int(n_streams), int(chunk), int(mem_budget), int(bytes_per_ray))
        h = C.c_void_p()
        N.check(N.lib().lt_server_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._keep = {}
        self._done = (N.lt_server_done * 256)()

    @property
    def handle(self):
        return self._h

    @staticmethod
    def prepare_map(m: Map, dtype: int, rays: Dict, out: Dict, n: int):
        """Marshal a map request once (the arguments of lt_server_submit_map);
        ``out`` is an empty_map_out(m.n_heads, n) dict."""
        torch = _torch()
        o = N.lt_map_out()
        for k in MAP_FIELDS:
            dt = torch.uint8 if k == "mask" else torch.float32
            setattr(o, k, _dev_ptr(out[k], dt, m.n_heads * n, f"out[{k}]") if n else None)
        return ("map", m.handle, int(dtype), _rays_struct(rays, n), o, int(n), (m, rays, out))

    @staticmethod
    def prepare_trace(lens: Lens, path, rays: Dict, out: Dict, n: int):
        """Marshal a trace request once; ``out`` is an empty_exit(n) dict."""
        torch = _torch()
        e = N.lt_exit()
        for k in EXIT_FIELDS:
            dt = torch.uint8 if k == "mask" else torch.float32
            setattr(e, k, _dev_ptr(out[k], dt, n, f"out[{k}]") if n else None)
        return ("trace", lens.handle, _path(path), _rays_struct(rays, n), e, int(n), (lens, rays, out))

    def submit(self, prepared, tag: int) -> None:
        """Queue a request marshalled by prepare_map / prepare_trace."""
        kind, h, arg, r, o, n, keep = prepared
        L = N.lib()
        if kind == "map":
            N.check(L.lt_server_submit_map(self._h, h, arg, C.byref(r), C.byref(o), n, int(tag)))
        else:
            N.check(L.lt_server_submit_trace(self._h, h, C.byref(arg), C.byref(r), C.byref(o), n,
                                             int(tag)))
        self._keep[int(tag)] = keep

    def submit_map(self, m: Map, dtype: int, rays: Dict, out: Dict, n: int, tag: int) -> None:
        """Queue lt_map_eval(m, dtype) of n rays into ``out`` (an
        empty_map_out(m.n_heads, n) dict); run lt_map_quantize(m, dtype) first."""
        self.submit(self.prepare_map(m, dtype, rays, out, n), tag)

    def submit_trace(self, lens: Lens, path, rays: Dict, out: Dict, n: int, tag: int) -> None:
        """Queue lt_trace(lens, path) of n rays into ``out`` (an empty_exit(n) dict)."""
        self.submit(self.prepare_trace(lens, path, rays, out, n), tag)

    def poll(self):
        """Advance the loop; returns ([(tag, done_s, status), ...], n_open)."""
        res = []
        n_open = C.c_int64()
        while True:
            k = C.c_int32()
            N.check(N.lib().lt_server_poll(self._h, self._done, len(self._done), C.byref(k),
                                           C.byref(n_open)))
            for i in range(k.value):
                d = self._done[i]
                self._keep.pop(int(d.tag), None)
                res.append((int(d.tag), float(d.done_s), int(d.status)))
            if k.value < len(self._done):
                return res, int(n_open.value)

    def stats(self):
        """(largest accounted in-flight bytes, launches so far)."""
        a, b = C.c_int64(), C.c_int64()
        N.check(N.lib().lt_server_stats(self._h, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def close(self):
        if self._h is not None and self._h.value:
            N.lib().lt_server_destroy(self._h)
        self._h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


LT_EVAL_MASK_ONLY, LT_EVAL_GATED = 1, 2


def lt_map_eval_ex(m: Map, dtype: int, rays: Dict, out: Optional[Dict] = None,
                   n: Optional[int] = None, flags: int = 0, mask_in=None, stream=None) -> Dict:
    """lt_map_eval with options: LT_EVAL_MASK_ONLY (logit and mask only) or
    LT_EVAL_GATED (exit fields only, valid where ``mask_in`` is set).
    ``out`` needs only the fields the call writes."""
    torch = _torch()
    if n is None:
        n = int(rays["x"].numel())
    if flags & LT_EVAL_GATED:
        wanted = MAP_FIELDS[2:]
    elif flags & LT_EVAL_MASK_ONLY:
        wanted = MAP_FIELDS[:2]
    else:
        wanted = MAP_FIELDS
    if out is None:
        full = empty_map_out(m.n_heads, n, rays["x"].device) if wanted == MAP_FIELDS else None
        out = full if full is not None else {
            k: torch.empty((m.n_heads, n), dtype=torch.uint8 if k == "mask" else torch.float32,
                           device=rays["x"].device) for k in wanted}
    o = N.lt_map_out()
    for k in MAP_FIELDS:
        if k not in wanted:
            setattr(o, k, None)
            continue
        dt = torch.uint8 if k == "mask" else torch.float32
        t = out[k]
        if n and (t.dim() != 2 or t.shape[0] != m.n_heads or t.shape[1] != n):
            raise ValueError(f"out[{k}] must have shape ({m.n_heads}, {n})")
        setattr(o, k, _dev_ptr(t, dt, m.n_heads * n, f"out[{k}]") if n else None)
    mp = None
    if flags & LT_EVAL_GATED:
        if mask_in is None:
            raise ValueError("LT_EVAL_GATED needs mask_in")
        mp = _dev_ptr(mask_in, torch.uint8, m.n_heads * n, "mask_in") if n else None
    N.check(N.lib().lt_map_eval_ex(m.handle, int(dtype), C.byref(_rays_struct(rays, n)), C.byref(o),
                                   int(n), int(flags), C.c_void_p(mp),
                                   C.c_void_p(_stream_ptr(stream) if n else 0)))
    return out


def lt_mask_index(mask, n: Optional[int] = None, capacity: Optional[int] = None, idx=None, count=None,
                  stream=None):
    """Dense list of the set entries of a uint8 mask (lt_mask_index), e.g. a
    classifier's mask: returns (idx int32 [capacity], count int64 [1]);
    entries past min(count, capacity) are not written."""
    torch = _torch()
    flat = mask.reshape(-1)
    if n is None:
        n = int(flat.numel())
    if capacity is None:
        capacity = n
    if idx is None:
        idx = torch.empty(max(capacity, 1), dtype=torch.int32, device=flat.device)
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=flat.device)
    mp = _dev_ptr(flat, torch.uint8, n, "mask") if n else None
    ip = _dev_ptr(idx, torch.int32, capacity, "idx") if capacity else None
    cp = _dev_ptr(count, torch.int64, 1, "count")
    N.check(N.lib().lt_mask_index(C.c_void_p(mp), int(n), C.c_void_p(ip), int(capacity), C.c_void_p(cp),
                                  C.c_void_p(_stream_ptr(stream))))
    return idx, count


def lt_map_eval_indexed(m: Map, dtype: int, rays: Dict, idx, count=None, max_n: Optional[int] = None,
                        out: Optional[Dict] = None, stream=None) -> Dict:
    """A one-head map on the listed rays (lt_map_eval_indexed): entry k below
    min(count, max_n) evaluates ray idx[k] and its exit fields land at k of
    the (1, max_n) outputs; ``count`` (int64 [1] on the device) may be None."""
    torch = _torch()
    if max_n is None:
        max_n = int(idx.numel())
    wanted = MAP_FIELDS[2:]
    if out is None:
        out = {k: torch.empty((1, max(max_n, 1)), dtype=torch.float32, device=rays["x"].device) for k in wanted}
    o = N.lt_map_out()
    for k in MAP_FIELDS:
        setattr(o, k, _dev_ptr(out[k], torch.float32, max_n, f"out[{k}]") if (k in wanted and max_n) else None)
    n_rays = int(rays["x"].numel())
    ip = _dev_ptr(idx, torch.int32, max_n, "idx") if max_n else None
    cp = _dev_ptr(count, torch.int64, 1, "count") if count is not None else None
    N.check(N.lib().lt_map_eval_indexed(m.handle, int(dtype), C.byref(_rays_struct(rays, n_rays)), C.c_void_p(ip),
                                        C.c_void_p(cp), int(max_n), C.byref(o),
                                        C.c_void_p(_stream_ptr(stream) if max_n else 0)))
    return out


COMPACT_FIELDS = ("x", "y", "dx", "dy", "dz", "throughput")


def lt_map_eval_compact(m: Map, dtype: int, rays: Dict, capacity: Optional[int] = None,
                        out: Optional[Dict] = None, n: Optional[int] = None, with_dz: bool = True,
                        with_bits: bool = True, stream=None) -> Dict:
    """Compacted evaluation (lt_map_eval_compact): per head the mask bitmap
    ``bits`` (int32 view of the uint32 words, shape (n_heads, ceil(n/32))),
    the valid rays' input indices ``idx`` and exit fields, shape
    (n_heads, capacity), and ``count`` (n_heads,) int64.  Entries of head p
    past count[p] (or capacity) are not written.  ``capacity`` defaults to n."""
    torch = _torch()
    if n is None:
        n = int(rays["x"].numel())
    if capacity is None:
        capacity = n
    dev = rays["x"].device
    P = m.n_heads
    words = (n + 31) // 32
    if out is None:
        out = {k: torch.empty((P, capacity), dtype=torch.float32, device=dev)
               for k in COMPACT_FIELDS if k != "dz" or with_dz}
        out["idx"] = torch.empty((P, capacity), dtype=torch.int32, device=dev)
        out["count"] = torch.empty(P, dtype=torch.int64, device=dev)
        if with_bits:
            out["bits"] = torch.empty((P, words), dtype=torch.int32, device=dev)
    o = N.lt_map_compact()
    cap_n = P * capacity
    for k in COMPACT_FIELDS:
        t = out.get(k)
        setattr(o, k, _dev_ptr(t, torch.float32, cap_n, f"out[{k}]") if (t is not None and cap_n) else None)
    o.idx = _dev_ptr(out["idx"], torch.int32, cap_n, "out[idx]") if cap_n else None
    o.mask_bits = (_dev_ptr(out["bits"], torch.int32, P * words, "out[bits]")
                   if (out.get("bits") is not None and n) else None)
    o.count = _dev_ptr(out["count"], torch.int64, P, "out[count]")
    o.capacity = int(capacity)
    N.check(N.lib().lt_map_eval_compact(m.handle, int(dtype), C.byref(_rays_struct(rays, n)),
                                        C.byref(o), int(n), C.c_void_p(_stream_ptr(stream))))
    return out


# -------------------------------------------------------------- training --

def lt_map_workspace_bytes(m: Map, n: int) -> int:
    return int(N.lib().lt_map_workspace_bytes(m.handle, int(n)))


def workspace(m: Map, n: int, device="cuda"):
    """A device workspace for training calls on n rays (torch allocations
    are 256-byte aligned)."""
    torch = _torch()
    ws = torch.empty(max(1, lt_map_workspace_bytes(m, n)), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def lt_map_forward_train(m: Map, rays: Dict, o_raw=None, ws=None, n: Optional[int] = None,
                         stream=None):
    """Training forward; returns (o_raw (6*n_heads, n) float32, workspace)."""
    torch = _torch()
    if n is None:
        n = int(rays["x"].numel())
    dev = rays["x"].device
    if o_raw is None:
        o_raw = torch.empty((6 * m.n_heads, n), dtype=torch.float32, device=dev)
    if ws is None:
        ws = workspace(m, n, dev)
    optr = _dev_ptr(o_raw, torch.float32, 6 * m.n_heads * n, "o_raw") if n else None
    N.check(N.lib().lt_map_forward_train(m.handle, C.byref(_rays_struct(rays, n)),
                                         C.c_void_p(optr), C.c_void_p(ws.data_ptr()),
                                         ws.numel(), int(n), C.c_void_p(_stream_ptr(stream))))
    return o_raw, ws


def lt_map_backward(m: Map, grad_o, ws, grad_params=None, n: Optional[int] = None, stream=None):
    """Hand-written backward of the last lt_map_forward_train on ``ws``."""
    torch = _torch()
    if n is None:
        n = int(grad_o.shape[-1])
    if grad_params is None:
        grad_params = torch.empty(m.n_params, dtype=torch.float32, device=grad_o.device)
    gptr = _dev_ptr(grad_o, torch.float32, 6 * m.n_heads * n, "grad_o") if n else grad_o.data_ptr()
    pptr = _dev_ptr(grad_params, torch.float32, m.n_params, "grad_params")
    N.check(N.lib().lt_map_backward(m.handle, C.c_void_p(gptr), C.c_void_p(ws.data_ptr()),
                                    ws.numel(), C.c_void_p(pptr), int(n),
                                    C.c_void_p(_stream_ptr(stream))))
    return grad_params


def lt_map_mark_updated(m: Map):
    """Tell the library that the map's parameters changed on the device
    outside its calls (a replayed training-step graph): the next evaluation
    repacks them."""
    N.check(N.lib().lt_map_mark_updated(m.handle))


def train_sched(device="cuda"):
    """A device lt_train_sched (16 bytes: float lr, int32 reserved, int64
    step) for cfg["sched"]: the training step then reads its learning rate
    and step count from device memory when it runs (graph replay)."""
    torch = _torch()
    return torch.zeros(16, dtype=torch.uint8, device=device)


def set_train_sched(sched, lr: float, step: int):
    """Write lr and step into a device lt_train_sched with two fill kernels
    on the current stream (ordered before later work on it, no host sync)."""
    sched.view(_torch().float32)[0].fill_(float(lr))
    sched.view(_torch().int64)[1].fill_(int(step))


def _train_args(m: Map, rays: Dict, targets: Dict, cfg: Dict, loss_out, n: Optional[int]):
    """Marshalled arguments of a fused training step."""
    torch = _torch()
    if n is None:
        n = int(rays["x"].numel())
    if loss_out is None:
        loss_out = torch.zeros(3, dtype=torch.float32, device=rays["x"].device)
    t = N.lt_targets()
    for k in TARGET_FIELDS:
        dt = torch.uint8 if k == "valid" else torch.float32
        setattr(t, k, _dev_ptr(targets[k], dt, m.n_heads * n, f"targets[{k}]"))
    sched = cfg.get("sched")
    sptr = None
    if sched is not None:
        assert sched.is_cuda and sched.dtype == torch.uint8 and sched.numel() == 16 and sched.is_contiguous(), \
            "cfg['sched'] must be a 16-byte device tensor from train_sched()"
        sptr = sched.data_ptr()
    c = N.lt_train_cfg(float(cfg.get("lr", 1e-3)), float(cfg.get("beta1", 0.9)),
                       float(cfg.get("beta2", 0.999)), float(cfg.get("eps", 1e-8)),
                       int(cfg.get("step", 1)), float(cfg.get("w_bce", 1.0)), float(cfg.get("w_l2", 1.0)),
                       float(cfg.get("w_cos", 0.0)), sptr)
    lp = C.c_void_p(_dev_ptr(loss_out, torch.float32, 3, "loss_out"))
    return n, _rays_struct(rays, n), t, c, loss_out, lp


def lt_map_train_step(m: Map, rays: Dict, targets: Dict, cfg: Dict, ws, loss_out=None,
                      n: Optional[int] = None, stream=None):
    """One fused forward + loss + backward + Adam step.  ``targets``: dict of
    (n_heads, n) CUDA tensors (valid uint8, the rest float32); ``cfg``: lr,
    beta1, beta2, eps, step (1-based), w_bce, w_l2, w_cos (cosine direction
    loss; 0 = squared error on all five outputs), sched (optional device
    lt_train_sched from train_sched(): lr and step are then read from it when
    the step runs).  Returns loss_out (device float32[3]: total, bce, l2)."""
    n, r, t, c, loss_out, lp = _train_args(m, rays, targets, cfg, loss_out, n)
    N.check(N.lib().lt_map_train_step(m.handle, C.byref(r), C.byref(t), int(n), C.byref(c),
                                      C.c_void_p(ws.data_ptr()), ws.numel(), lp,
                                      C.c_void_p(_stream_ptr(stream))))
    return loss_out


def lt_map_train_step_static(m: Map, rays: Dict, targets: Dict, cfg: Dict, loss_out=None,
                             n: Optional[int] = None, stream=None):
    """lt_map_train_step with the workspace taken from the library's static
    per-GPU scratch (no allocation in the call; batches whose workspace
    exceeds LT_STATIC_SCRATCH_BYTES raise).  Overlapping calls on one GPU
    race on that scratch."""
    n, r, t, c, loss_out, lp = _train_args(m, rays, targets, cfg, loss_out, n)
    N.check(N.lib().lt_map_train_step_static(m.handle, C.byref(r), C.byref(t), int(n), C.byref(c),
                                             lp, C.c_void_p(_stream_ptr(stream))))
    return loss_out


def lt_map_adam_state(m: Map, mv=None, to_map: bool = False, stream=None):
    """Get (to_map=False) or set (True) the Adam moments as a (2, n_params)
    float32 CUDA tensor."""
    torch = _torch()
    if mv is None:
        mv = torch.empty((2, m.n_params), dtype=torch.float32, device="cuda")
    _dev_ptr(mv, torch.float32, 2 * m.n_params, "mv")
    N.check(N.lib().lt_map_adam_state(m.handle, C.c_void_p(mv[0].data_ptr()),
                                      C.c_void_p(mv[1].data_ptr()), m.n_params, int(to_map),
                                      C.c_void_p(_stream_ptr(stream))))
    return mv
