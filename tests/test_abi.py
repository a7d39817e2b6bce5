"""The C-ABI library loads, exports every symbol include/lt.h declares, and
its host-side logic (validation, error codes, path bookkeeping) behaves as
documented.  No GPU work is launched here."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2605_04017_amd as lt
import synth
from paper_2605_04017_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "lt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lt_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_header_symbols():
    names = header_functions()
    assert "lt_trace" in names and "lt_lens_create" in names
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (lt_[a-z0-9_]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = N.lib()
    for n in names:
        assert hasattr(L, n)
    # the binding declares a signature for every header function
    assert set(names) <= set(N.SIGNATURES)


def test_status_strings():
    L = N.lib()
    assert L.lt_status_str(0) == b"LT_OK"
    assert L.lt_status_str(2) == b"LT_ERR_LENS"
    assert L.lt_version() >= 100


def test_lens_create_and_query():
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    assert (h.n_surfaces, h.n_refracting, h.n_ghost_paths) == (12, 11, 55)
    assert lt.lt_lens_query(h)[:3] == (12, 11, 55)
    h.close()


def _abcd_reduced(lens, lam_nm):
    """System matrix (heights, reduced angles) from the front vertex to the
    last vertex: refraction [[1, 0], [-P, 1]] with P = (n' - n) / R, transfer
    [[1, t / n'], [0, 1]] (a product of matrices; the library traces y-nu)."""
    import numpy as np
    import oracle
    ns = [1.0] + [oracle.glass_index(lens, s.glass_after, lam_nm) for s in lens.surfaces]
    M = np.eye(2)
    for k, s in enumerate(lens.surfaces):
        P = 0.0 if s.radius == 0 else (ns[k + 1] - ns[k]) / s.radius
        M = np.array([[1.0, 0.0], [-P, 1.0]]) @ M
        if k < len(lens.surfaces) - 1:
            M = np.array([[1.0, s.thickness / ns[k + 1]], [0.0, 1.0]]) @ M
    return M, ns[-1]


@pytest.mark.parametrize("config", [1, 2, 5])
def test_lens_paraxial_focal_lengths(config):
    """lt_lens_query / lt_lens_paraxial EFL and back focal distance against
    the ABCD matrix of the prescription (EFL = -1/C, BFD = -n' A/C), which the
    oracle pins tie to finite-height traces of the exact tracer; and the
    synthetic lenses put the sensor at the d-line paraxial focus."""
    lenses = [synth.config_lens(config)] if config != 5 else synth.serve_lenses()
    for lens in lenses:
        h = lt.lt_lens_create(lens.surfaces, lens.glasses)
        for lam in (587.5618, 450.0, 650.0):
            M, n_img = _abcd_reduced(lens, lam)
            efl, bfl = lt.lt_lens_paraxial(h, lam)
            assert abs(efl - (-1.0 / M[1, 0])) <= 1e-12 * abs(efl)
            assert abs(bfl - (-n_img * M[0, 0] / M[1, 0])) <= 1e-12 * abs(bfl)
        ns_, nr, ng, efl_d, bfl_d = lt.lt_lens_query(h)
        assert (efl_d, bfl_d) == lt.lt_lens_paraxial(h, 587.5618)
        assert abs(bfl_d - lens.surfaces[-1].thickness) < 1e-6 * abs(bfl_d)
        with pytest.raises(lt.LtError):
            lt.lt_lens_paraxial(h, 200.0)
        h.close()


@pytest.mark.parametrize("mutate,msg", [
    (lambda s, g: s[0].__setattr__("thickness", -1.0), "negative thickness"),
    (lambda s, g: s[0].__setattr__("semi_diameter", 0.0), "semi-diameter"),
    (lambda s, g: s[0].__setattr__("semi_diameter", abs(s[0].radius) * 1.01), "smaller than"),
    (lambda s, g: s[0].__setattr__("glass_after", 99), "glass index"),
    (lambda s, g: s[5].__setattr__("radius", 50.0), "flat"),
    (lambda s, g: s[1].__setattr__("is_stop", 1), "stop"),
    (lambda s, g: g[1].coef.__setitem__(0, 0.2), "index not real"),
])
def test_lens_validation(mutate, msg):
    import copy
    lens = copy.deepcopy(synth.config_lens(2))
    mutate(lens.surfaces, lens.glasses)
    with pytest.raises(lt.LtError) as e:
        lt.lt_lens_create(lens.surfaces, lens.glasses)
    assert e.value.status in (N.LT_ERR_LENS, N.LT_ERR_ARG)
    assert msg in str(e.value)


def test_lens_limits():
    lens = synth.config_lens(1)
    with pytest.raises(lt.LtError) as e:
        lt.lt_lens_create([], lens.glasses)
    assert e.value.status == N.LT_ERR_ARG
    too_many = [lens.surfaces[1]] * (N.LT_MAX_SURFACES + 1)
    with pytest.raises(lt.LtError):
        lt.lt_lens_create(too_many, lens.glasses)


def test_ghost_index_roundtrip():
    for n in (2, 3, 11, 22):
        seen = set()
        for j in range(1, n + 1):
            for i in range(j + 1, n + 1):
                k = lt.lt_ghost_index(n, j, i)
                assert 0 <= k < n * (n - 1) // 2
                assert lt.lt_ghost_path(n, k) == (1, j, i)
                seen.add(k)
        assert len(seen) == n * (n - 1) // 2
    assert lt.lt_ghost_index(11, 3, 3) == -1
    with pytest.raises(lt.LtError):
        lt.lt_ghost_path(11, 55)


def test_trace_argument_errors_without_gpu():
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    L = N.lib()
    rays, ex = N.lt_rays(), N.lt_exit()
    # bad path is reported before any device work
    p = N.lt_path(1, 5, 5)
    assert L.lt_trace(h.handle, C.byref(p), C.byref(rays), C.byref(ex), 10, None) == N.LT_ERR_PATH
    p = N.lt_path(0, 0, 0)
    # n = 0 is a no-op, negative n and NULL fields are argument errors
    assert L.lt_trace(h.handle, C.byref(p), C.byref(rays), C.byref(ex), 0, None) == N.LT_OK
    assert L.lt_trace(h.handle, C.byref(p), C.byref(rays), C.byref(ex), -1, None) == N.LT_ERR_ARG
    assert L.lt_trace(h.handle, C.byref(p), C.byref(rays), C.byref(ex), 5, None) == N.LT_ERR_ARG
    assert b"NULL" in L.lt_last_error()
    assert L.lt_trace(None, C.byref(p), C.byref(rays), C.byref(ex), 5, None) == N.LT_ERR_ARG
    assert L.lt_trace_ex(h.handle, C.byref(p), C.byref(rays), C.byref(ex), 0, 0x80, None) == N.LT_ERR_ARG


@pytest.mark.parametrize("desc", [(5, 128, 5, 1, 0), (6, 100, 5, 1, 0), (6, 128, 0, 1, 0),
                                  (6, 128, 9, 1, 0), (6, 128, 5, 0, 0), (6, 128, 5, 65, 0),
                                  (6, 128, 5, 1, 7), (6, 128, 5, 1, 0, 2),
                                  (6, 128, 5, 1, 0, 0, 3)])
def test_map_desc_validation(desc):
    """Bad shapes are rejected before any device allocation."""
    d = N.lt_map_desc(*desc)
    h = C.c_void_p()
    assert N.lib().lt_map_create(C.byref(d), C.byref(h)) == N.LT_ERR_ARG
    assert h.value is None


def test_map_null_handles():
    L = N.lib()
    assert L.lt_map_num_params(None) == -1
    assert L.lt_map_eval(None, 1, None, None, 0, None) == N.LT_ERR_ARG
    assert L.lt_map_destroy(None) == N.LT_OK


def test_splat_and_forward_raygen_argument_errors_without_gpu():
    """Argument validation of lt_splat and lt_rays_generate_forward happens
    before any device call (n = 0 is a no-op)."""
    L = N.lib()
    s = N.lt_sensor(36.0, 24.0, 480, 320)
    assert L.lt_splat(None, None, None, None, None, 0, 1, C.byref(s), 1.0, None, None) == N.LT_OK
    assert L.lt_splat(None, None, None, None, None, 5, 5, C.byref(s), 1.0, None, None) == N.LT_ERR_ARG
    assert L.lt_splat(None, None, None, None, None, -1, 5, C.byref(s), 1.0, None, None) == N.LT_ERR_ARG
    assert L.lt_splat(None, None, None, None, None, 0, 0, C.byref(s), 1.0, None, None) == N.LT_ERR_ARG
    assert L.lt_splat(None, None, None, None, None, 0, 1, None, 1.0, None, None) == N.LT_ERR_ARG
    for bad in ((0.0, 24.0, 480, 320), (36.0, 24.0, 0, 320), (36.0, float("inf"), 480, 320),
                (36.0, 24.0, 1 << 16, 1 << 16), (36.0, 24.0, 480, -3)):
        sb = N.lt_sensor(*bad)
        assert L.lt_splat(None, None, None, None, None, 0, 1, C.byref(sb), 1.0, None, None) == N.LT_ERR_ARG
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    b = N.lt_ray_buffers()

    def gen(light, at_inf, ap=10.0, lam=(400.0, 700.0), n=0):
        cfg = N.lt_raygen_forward(1, 0, (C.c_float * 3)(*light), at_inf, ap, *lam)
        return L.lt_rays_generate_forward(h.handle, C.byref(cfg), C.byref(b), n, None)
    assert gen((0.0, 0.0, 1.0), 1) == N.LT_OK
    assert gen((0.0, 0.0, 1.0), 1, n=4) == N.LT_ERR_ARG          # NULL outputs
    assert gen((0.0, 0.0, 1.0), 1, n=-1) == N.LT_ERR_ARG
    assert gen((0.0, 0.0, -1.0), 1) == N.LT_ERR_ARG               # travels away from the lens
    assert gen((0.0, 0.0, 0.0), 1) == N.LT_ERR_ARG
    assert gen((0.0, 0.0, 3.0), 0) == N.LT_ERR_ARG                # light behind the input plane
    assert gen((0.0, 0.0, -100.0), 0) == N.LT_OK
    assert gen((0.0, 0.0, 1.0), 1, ap=0.0) == N.LT_ERR_ARG
    assert gen((0.0, 0.0, 1.0), 1, lam=(700.0, 400.0)) == N.LT_ERR_ARG


def test_splat_wrapper_empty_without_gpu():
    import torch
    e = torch.empty(0, dtype=torch.float32)
    img = lt.lt_splat(e, e, e, e, (36.0, 24.0, 48, 32))
    assert img.shape == (1, 32, 48) and float(img.abs().sum()) == 0.0


def test_mcmc_argument_errors_without_gpu():
    L = N.lib()
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    st = N.lt_mcmc_state()
    p = N.lt_path(1, 2, 10)

    def cfg(**kw):
        a = dict(seed=1, first_step=0, half_width_mm=18.0, half_height_mm=12.0, lambda_min_nm=400.0,
                 lambda_max_nm=700.0, lambda_mode=0, p_large=0.1, target_accept=0.234)
        a.update(kw)
        return N.lt_mcmc_cfg(*a.values())

    def run(c, n=0, steps=4, path=p):
        return L.lt_mcmc_run(h.handle, C.byref(path), C.byref(c), C.byref(st), n, steps, None, None,
                             None, 0, None)
    assert run(cfg()) == N.LT_OK                                   # no chains: no-op
    assert run(cfg(), n=8) == N.LT_ERR_ARG                         # NULL state fields
    assert run(cfg(), n=-1) == N.LT_ERR_ARG
    assert run(cfg(p_large=1.5)) == N.LT_ERR_ARG
    assert run(cfg(target_accept=0.0)) == N.LT_ERR_ARG
    assert run(cfg(lambda_mode=3)) == N.LT_ERR_ARG
    assert run(cfg(lambda_mode=1, lambda_max_nm=400.0)) == N.LT_ERR_ARG
    assert run(cfg(half_width_mm=0.0)) == N.LT_ERR_ARG
    assert run(cfg(), path=N.lt_path(1, 3, 3)) == N.LT_ERR_PATH
    assert L.lt_mcmc_run(h.handle, C.byref(p), C.byref(cfg()), C.byref(st), 0, 1, None, None, None, 8,
                         None) == N.LT_ERR_ARG                      # unknown flag
    assert L.lt_mcmc_init(C.byref(st), 0, C.c_float(0.05), None) == N.LT_OK
    assert L.lt_mcmc_init(C.byref(st), 4, C.c_float(0.05), None) == N.LT_ERR_ARG
    assert L.lt_mcmc_init(C.byref(st), 0, C.c_float(0.9), None) == N.LT_ERR_ARG
    rg = N.lt_raygen(1, 0, 18.0, 12.0, 400.0, 700.0, 2)
    b = N.lt_ray_buffers()
    assert L.lt_rays_generate(h.handle, C.byref(rg), C.byref(b), 0, None) == N.LT_ERR_ARG


def test_contradictory_trace_flags_rejected_without_gpu():
    L = N.lib()
    lens = synth.config_lens(1)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    p = N.lt_path(0, 0, 0)
    rays, ex = N.lt_rays(), N.lt_exit()
    both = N.LT_TRACE_FP64 | N.LT_TRACE_PLAIN_FP32
    assert L.lt_trace_ex(h.handle, C.byref(p), C.byref(rays), C.byref(ex), 0, both, None) == N.LT_ERR_ARG
    assert L.lt_trace_ex(h.handle, C.byref(p), C.byref(rays), C.byref(ex), 0, N.LT_TRACE_FP64, None) == N.LT_OK


def test_server_argument_errors_without_gpu():
    """The serving loop validates its configuration and handles before any
    HIP call (no device here)."""
    L = N.lib()
    h = C.c_void_p()
    for bad in ((0, 1, 1, 0), (17, 1, 1, 0), (4, 0, 1, 0), (4, 1, 0, 0), (4, 1, 1, -1)):
        assert L.lt_server_create(C.byref(N.lt_server_cfg(*bad)), C.byref(h)) == N.LT_ERR_ARG
        assert "LT_ERR_ARG" in L.lt_last_error().decode()
    assert L.lt_server_create(None, C.byref(h)) == N.LT_ERR_ARG
    assert L.lt_server_destroy(None) == N.LT_OK
    k, n_open = C.c_int32(), C.c_int64()
    assert L.lt_server_poll(None, None, 0, C.byref(k), C.byref(n_open)) == N.LT_ERR_ARG
    assert L.lt_server_stats(None, None, None) == N.LT_ERR_ARG
    rays, mo, ex, p = N.lt_rays(), N.lt_map_out(), N.lt_exit(), N.lt_path(0, 0, 0)
    assert L.lt_server_submit_map(None, None, 1, C.byref(rays), C.byref(mo), 0, 0) == N.LT_ERR_ARG
    assert L.lt_server_submit_trace(None, None, C.byref(p), C.byref(rays), C.byref(ex), 0,
                                    0) == N.LT_ERR_ARG
