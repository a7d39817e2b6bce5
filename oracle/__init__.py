"""FP64 CPU oracle for the lens transport hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg are the only callers.  Nothing here is used by, or uses, the HIP
implementation in ``paper_2605_04017_amd``.

* ``lt_oracle.c``  -- sequential FP64 ray tracer (Sec. 3 operators p, d, f and
  their composition), built with gcc into ``liblt_oracle.so``;
* ``mlp.py``        -- FP64 reference of the factorised classifier/regressor
  network (Sec. 4.2), its loss, gradient, Adam step and the BF16/FP8 rounding
  the GPU path applies.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lt_oracle.c")
_LIB = os.path.join(_HERE, "liblt_oracle.so")
_lib = None


class OrSurface(C.Structure):
    _fields_ = [("radius", C.c_double), ("thickness", C.c_double), ("sd", C.c_double),
                ("glass_after", C.c_int32), ("is_stop", C.c_int32)]


class OrGlass(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("coef", C.c_double * 6)]


class OrStep(C.Structure):
    _fields_ = [("surf", C.c_int32), ("type", C.c_int32), ("dir", C.c_int32), ("pad", C.c_int32)]


class OrDiag(C.Structure):
    _fields_ = [("edge_margin", C.c_double), ("tir_margin", C.c_double),
                ("graze_margin", C.c_double), ("fail_step", C.c_int32), ("fail_kind", C.c_int32)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        L.or_build_sequence.argtypes = [P(OrSurface), C.c_int, C.c_int, C.c_int, C.c_int,
                                        P(OrStep), C.c_int]
        L.or_build_sequence.restype = C.c_int
        L.or_trace_sequence.argtypes = [P(OrSurface), C.c_int, P(OrGlass), C.c_int, P(OrStep),
                                        C.c_int, C.c_double, P(C.c_double), P(C.c_double),
                                        C.c_double, C.c_int, P(C.c_double), P(C.c_double),
                                        P(C.c_double), P(OrDiag)]
        L.or_trace_sequence.restype = C.c_int
        L.or_trace_batch.argtypes = ([P(OrSurface), C.c_int, P(OrGlass), C.c_int, C.c_int, C.c_int,
                                      C.c_int, C.c_int, C.c_int64] + [C.c_void_p] * 6 + [C.c_void_p]
                                     + [C.c_void_p] * 7 + [C.c_void_p] * 4 + [C.c_int])
        L.or_trace_batch.restype = C.c_int64
        L.or_forward_plane_z.argtypes = [P(OrSurface), C.c_int]
        L.or_forward_plane_z.restype = C.c_double
        L.or_glass_index.argtypes = [P(OrGlass), C.c_int, C.c_int, C.c_double]
        L.or_glass_index.restype = C.c_double
        _lib = L
    return _lib


def _pack(lens):
    ns = len(lens.surfaces)
    S = (OrSurface * ns)()
    for k, s in enumerate(lens.surfaces):
        S[k].radius = s.radius
        S[k].thickness = s.thickness
        S[k].sd = s.semi_diameter
        S[k].glass_after = s.glass_after
        S[k].is_stop = s.is_stop
    ng = len(lens.glasses)
    G = (OrGlass * ng)()
    for k, g in enumerate(lens.glasses):
        G[k].kind = g.kind
        for m in range(6):
            G[k].coef[m] = g.coef[m]
    return S, ns, G, ng


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def trace(lens, rays: dict, path=(0, 0, 0), nthreads: int = 0, diag: bool = False,
          forward: bool = False) -> dict:
    """Trace sensor-side FP32 rays through ``lens`` along ``path`` = (kind, j, i).

    kind 0 = transmit, kind 1 = two-reflection ghost with 1-based refracting
    surface indices j < i.  Returns FP64 arrays: mask, x, y, z (= 0, the output
    plane), dx, dy, dz, throughput; with ``diag`` also edge/TIR/grazing margins
    and the failure kind.  nthreads = 0 uses OpenMP's default.

    forward: the rays start on the forward input plane (``forward_plane_z``)
    travelling toward the image and follow the path's interactions in reverse
    order (forward light tracing, Sec. 3); the outputs lie on the sensor plane.
    """
    L = lib()
    S, ns, G, ng = _pack(lens)
    n = int(rays["x"].shape[0])
    f = {k: np.ascontiguousarray(rays[k], dtype=np.float32) for k in
         ("x", "y", "dx", "dy", "dz", "lambda_nm")}
    out = {"mask": np.zeros(n, np.uint8)}
    for k in ("x", "y", "z", "dx", "dy", "dz", "throughput"):
        out[k] = np.empty(n, np.float64)
    dg = {}
    if diag:
        for k in ("edge_margin", "tir_margin", "graze_margin"):
            dg[k] = np.empty(n, np.float64)
        dg["fail_kind"] = np.empty(n, np.int32)
    nv = L.or_trace_batch(S, ns, G, ng, int(path[0]), int(path[1]), int(path[2]), int(bool(forward)), n,
                          _ptr(f["x"]), _ptr(f["y"]), _ptr(f["dx"]), _ptr(f["dy"]),
                          _ptr(f["dz"]), _ptr(f["lambda_nm"]), _ptr(out["mask"]),
                          _ptr(out["x"]), _ptr(out["y"]), _ptr(out["z"]), _ptr(out["dx"]),
                          _ptr(out["dy"]), _ptr(out["dz"]), _ptr(out["throughput"]),
                          _ptr(dg.get("edge_margin")), _ptr(dg.get("tir_margin")),
                          _ptr(dg.get("graze_margin")), _ptr(dg.get("fail_kind")),
                          int(nthreads))
    if nv < 0:
        raise ValueError(f"invalid path {path}")
    out.update(dg)
    out["n_valid"] = int(nv)
    return out


def forward_plane_z(lens) -> float:
    """z of the forward input plane (1 mm in front of the first surface's
    foremost point within its clear aperture)."""
    S, ns, _, _ = _pack(lens)
    return float(lib().or_forward_plane_z(S, ns))


def build_sequence(lens, kind: int, j: int = 0, i: int = 0):
    """Interaction sequence of a path as a list of (surface, type, dir)."""
    L = lib()
    S, ns, _, _ = _pack(lens)
    buf = (OrStep * 256)()
    m = L.or_build_sequence(S, ns, kind, j, i, buf, 256)
    if m < 0:
        raise ValueError("invalid path")
    return [(buf[k].surf, buf[k].type, buf[k].dir) for k in range(m)]


def trace_sequence(lens, seq, lam_nm: float, origin, direction, z_out: float, exit_dir: int):
    """Trace one FP64 ray from a global origin along an explicit sequence.

    Returns (valid, position[3], direction[3], throughput, diag dict).
    """
    L = lib()
    S, ns, G, ng = _pack(lens)
    m = len(seq)
    buf = (OrStep * max(1, m))()
    for k, (sf, ty, dr) in enumerate(seq):
        buf[k].surf, buf[k].type, buf[k].dir = sf, ty, dr
    o = (C.c_double * 3)(*origin)
    d = (C.c_double * 3)(*direction)
    P = (C.c_double * 3)()
    D = (C.c_double * 3)()
    I = C.c_double()
    dg = OrDiag()
    ok = L.or_trace_sequence(S, ns, G, ng, buf, m, float(lam_nm), o, d, float(z_out),
                             int(exit_dir), P, D, C.byref(I), C.byref(dg))
    return (bool(ok), np.array(P[:]), np.array(D[:]), I.value,
            {"edge_margin": dg.edge_margin, "tir_margin": dg.tir_margin,
             "graze_margin": dg.graze_margin, "fail_step": dg.fail_step,
             "fail_kind": dg.fail_kind})


def glass_index(lens, gi: int, lam_nm: float) -> float:
    L = lib()
    _, _, G, ng = _pack(lens)
    return L.or_glass_index(G, ng, gi, float(lam_nm))
