"""ctypes declarations of liblt.so (include/lt.h).  Loading fails loudly if the
library has not been built: there is no fallback implementation."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblt.so")

LT_OK, LT_ERR_ARG, LT_ERR_LENS, LT_ERR_PATH, LT_ERR_DTYPE, LT_ERR_OOM, LT_ERR_DEVICE, \
    LT_ERR_STATE = range(8)
LT_MAX_SURFACES = 24
LT_MAX_GLASSES = 24
LT_TRACE_PLAIN_FP32 = 1
LT_TRACE_FORWARD = 2
LT_TRACE_FP64 = 4
LT_LAMBDA_UNIFORM, LT_LAMBDA_CIE = 0, 1


class LtError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


class lt_glass(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("coef", C.c_double * 6)]


class lt_surface(C.Structure):
    _fields_ = [("radius_mm", C.c_double), ("thickness_mm", C.c_double),
                ("semi_diameter_mm", C.c_double), ("glass_after", C.c_int32),
                ("is_stop", C.c_int32)]


class lt_path(C.Structure):
    _fields_ = [("kind", C.c_int32), ("j", C.c_int32), ("i", C.c_int32)]


class lt_rays(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "dx", "dy", "dz", "lambda_nm")]


class lt_ray_buffers(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "dx", "dy", "dz", "lambda_nm")]


class lt_raygen(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("first", C.c_uint64), ("half_width_mm", C.c_float),
                ("half_height_mm", C.c_float), ("lambda_min_nm", C.c_float),
                ("lambda_max_nm", C.c_float), ("lambda_mode", C.c_int32)]


class lt_mcmc_cfg(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("first_step", C.c_uint64), ("half_width_mm", C.c_float),
                ("half_height_mm", C.c_float), ("lambda_min_nm", C.c_float),
                ("lambda_max_nm", C.c_float), ("lambda_mode", C.c_int32), ("p_large", C.c_float),
                ("target_accept", C.c_float)]


class lt_mcmc_state(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("u", "step", "n_small", "visible")]


class lt_raygen_forward(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("first", C.c_uint64), ("light", C.c_float * 3),
                ("at_infinity", C.c_int32), ("aperture_mm", C.c_float),
                ("lambda_min_nm", C.c_float), ("lambda_max_nm", C.c_float)]


class lt_sensor(C.Structure):
    _fields_ = [("width_mm", C.c_float), ("height_mm", C.c_float), ("nx", C.c_int32),
                ("ny", C.c_int32)]


class lt_exit(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("mask", "x", "y", "dx", "dy", "dz", "throughput")]


class lt_map_desc(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32),
                ("n_heads", C.c_int32), ("activation", C.c_int32), ("canonical", C.c_int32),
                ("forward", C.c_int32)]


class lt_map_out(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("logit", "mask", "x", "y", "dx", "dy", "dz",
                                           "throughput")]


class lt_map_compact(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("mask_bits", "idx", "x", "y", "dx", "dy", "dz",
                                           "throughput", "count")] + [("capacity", C.c_int64)]


class lt_targets(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("valid", "x", "y", "dx", "dy", "throughput")]


class lt_train_cfg(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int64), ("w_bce", C.c_float), ("w_l2", C.c_float), ("w_cos", C.c_float),
                ("sched", C.c_void_p)]


class lt_train_sched(C.Structure):
    _fields_ = [("lr", C.c_float), ("reserved", C.c_int32), ("step", C.c_int64)]


class lt_server_cfg(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("chunk", C.c_int64), ("mem_budget", C.c_int64),
                ("bytes_per_ray", C.c_int64)]


class lt_server_done(C.Structure):
    _fields_ = [("tag", C.c_int64), ("done_s", C.c_double), ("status", C.c_int32)]


LT_F32, LT_BF16, LT_FP8 = 0, 1, 2
LT_ACT_TANH, LT_ACT_RELU = 0, 1

_lib = None

# name -> (restype, argtypes); every exported symbol of include/lt.h
SIGNATURES = {
    "lt_status_str": (C.c_char_p, [C.c_int]),
    "lt_last_error": (C.c_char_p, []),
    "lt_version": (C.c_int32, []),
    "lt_lens_create": (C.c_int, [C.POINTER(lt_surface), C.c_int32, C.POINTER(lt_glass),
                                 C.c_int32, C.POINTER(C.c_void_p)]),
    "lt_lens_destroy": (C.c_int, [C.c_void_p]),
    "lt_lens_query": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lt_lens_paraxial": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]),
    "lt_canonical_frame": (C.c_int, [C.POINTER(lt_rays), C.POINTER(lt_ray_buffers), C.POINTER(lt_exit),
                                     C.c_int32, C.c_int64, C.c_void_p]),
    "lt_lens_planes": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "lt_ghost_index": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32]),
    "lt_ghost_path": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(lt_path)]),
    "lt_path_encode": (C.c_int, [C.c_int32, C.POINTER(lt_path), C.POINTER(C.c_uint64)]),
    "lt_path_decode": (C.c_int, [C.c_int32, C.c_uint64, C.POINTER(lt_path)]),
    "lt_trace_compact": (C.c_int, [C.c_void_p, C.POINTER(lt_path), C.POINTER(lt_rays),
                                   C.POINTER(lt_exit), C.c_void_p, C.c_void_p, C.c_int64,
                                   C.c_uint32, C.c_void_p]),
    "lt_map_quantize": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "lt_map_eval_ex": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(lt_rays), C.POINTER(lt_map_out),
                                 C.c_int64, C.c_uint32, C.c_void_p, C.c_void_p]),
    "lt_map_eval_compact": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(lt_rays),
                                      C.POINTER(lt_map_compact), C.c_int64, C.c_void_p]),
    "lt_mask_index": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "lt_map_eval_indexed": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(lt_rays), C.c_void_p, C.c_void_p,
                                      C.c_int64, C.POINTER(lt_map_out), C.c_void_p]),
    "lt_rays_generate": (C.c_int, [C.c_void_p, C.POINTER(lt_raygen), C.POINTER(lt_ray_buffers),
                                   C.c_int64, C.c_void_p]),
    "lt_rays_generate_forward": (C.c_int, [C.c_void_p, C.POINTER(lt_raygen_forward),
                                           C.POINTER(lt_ray_buffers), C.c_int64, C.c_void_p]),
    "lt_mcmc_init": (C.c_int, [C.POINTER(lt_mcmc_state), C.c_int64, C.c_float, C.c_void_p]),
    "lt_mcmc_run": (C.c_int, [C.c_void_p, C.POINTER(lt_path), C.POINTER(lt_mcmc_cfg),
                              C.POINTER(lt_mcmc_state), C.c_int64, C.c_int32,
                              C.POINTER(lt_ray_buffers), C.POINTER(lt_exit), C.c_void_p, C.c_uint32,
                              C.c_void_p]),
    "lt_splat": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                           C.c_int64, C.POINTER(lt_sensor), C.c_float, C.c_void_p, C.c_void_p]),
    "lt_server_create": (C.c_int, [C.POINTER(lt_server_cfg), C.POINTER(C.c_void_p)]),
    "lt_server_destroy": (C.c_int, [C.c_void_p]),
    "lt_server_submit_map": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(lt_rays),
                                       C.POINTER(lt_map_out), C.c_int64, C.c_int64]),
    "lt_server_submit_trace": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(lt_path),
                                         C.POINTER(lt_rays), C.POINTER(lt_exit), C.c_int64,
                                         C.c_int64]),
    "lt_server_poll": (C.c_int, [C.c_void_p, C.POINTER(lt_server_done), C.c_int32,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "lt_server_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "lt_trace": (C.c_int, [C.c_void_p, C.POINTER(lt_path), C.POINTER(lt_rays),
                           C.POINTER(lt_exit), C.c_int64, C.c_void_p]),
    "lt_trace_ex": (C.c_int, [C.c_void_p, C.POINTER(lt_path), C.POINTER(lt_rays),
                              C.POINTER(lt_exit), C.c_int64, C.c_uint32, C.c_void_p]),
    "lt_map_create": (C.c_int, [C.POINTER(lt_map_desc), C.POINTER(C.c_void_p)]),
    "lt_map_destroy": (C.c_int, [C.c_void_p]),
    "lt_map_num_params": (C.c_int64, [C.c_void_p]),
    "lt_map_set_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "lt_map_get_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "lt_map_mark_updated": (C.c_int, [C.c_void_p]),
    "lt_map_set_norm": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                  C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "lt_map_eval": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(lt_rays), C.POINTER(lt_map_out),
                              C.c_int64, C.c_void_p]),
    "lt_map_workspace_bytes": (C.c_int64, [C.c_void_p, C.c_int64]),
    "lt_map_forward_train": (C.c_int, [C.c_void_p, C.POINTER(lt_rays), C.c_void_p, C.c_void_p,
                                       C.c_int64, C.c_int64, C.c_void_p]),
    "lt_map_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_int64, C.c_void_p]),
    "lt_map_train_step": (C.c_int, [C.c_void_p, C.POINTER(lt_rays), C.POINTER(lt_targets),
                                    C.c_int64, C.POINTER(lt_train_cfg), C.c_void_p, C.c_int64,
                                    C.c_void_p, C.c_void_p]),
    "lt_map_train_step_static": (C.c_int, [C.c_void_p, C.POINTER(lt_rays), C.POINTER(lt_targets),
                                           C.c_int64, C.POINTER(lt_train_cfg), C.c_void_p,
                                           C.c_void_p]),
    "lt_map_adam_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                    C.c_void_p]),
}

# Bytes of the library's static training scratch per GPU (include/lt.h).
LT_STATIC_SCRATCH_BYTES = 64 << 20


def lib():
    """The loaded liblt.so; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2605_04017_amd.build` "
                              "(there is no non-HIP fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != LT_OK:
        msg = lib().lt_last_error().decode()
        raise LtError(status, msg)
