"""GPU parity of the brute-force tracer (lt_trace) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth

from parity import compare_trace, to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _to_dev(rays, dev):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in rays.items()}


def _gpu_trace(lens, rays, dev, path=(0, 0, 0), flags=0):
    import torch
    import paper_2605_04017_amd as lt
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    r = _to_dev(rays, dev)
    n = int(rays["x"].shape[0])
    out = lt.empty_exit(n, dev)
    if flags:
        lt.lt_trace_ex(h, path, r, out, n, flags)
    else:
        lt.lt_trace(h, path, r, out, n)
    torch.cuda.synchronize()
    return to_numpy(out)


def _report(name, st):
    print(f"[parity] {name}: {st}", flush=True)


def test_c1_doublet_full(dev):
    """Cemented doublet + stop, 65,536 rays: transmit and all three ghosts."""
    L = synth.config_lens(1)
    rays = synth.config_rays(1)
    for path in [(0, 0, 0), (1, 1, 2), (1, 1, 3), (1, 2, 3)]:
        st = compare_trace(_gpu_trace(L, rays, dev, path), oracle.trace(L, rays, path, diag=True))
        _report(f"C1 {path}", st)
        assert st["valid"] > 1000


def test_c2_double_gauss_full_size(dev):
    """11-surface lens, 4,194,304 rays (the benchmark workload), transmit,
    every ray compared."""
    L = synth.config_lens(2)
    rays = synth.config_rays(2)
    st = compare_trace(_gpu_trace(L, rays, dev), oracle.trace(L, rays, diag=True))
    _report("C2 transmit 4M", st)
    assert st["valid"] > 500000


def test_c2_all_55_ghosts(dev):
    L = synth.config_lens(2)
    rays = synth.config_rays(2, 131072)
    worst = 0.0
    for j in range(1, 12):
        for i in range(j + 1, 12):
            st = compare_trace(_gpu_trace(L, rays, dev, (1, j, i)),
                               oracle.trace(L, rays, (1, j, i), diag=True))
            worst = max(worst, st.get("pos_max", 0.0))
    print(f"[parity] C2 55 ghosts worst position error {worst:.3e} mm", flush=True)


def test_c3_size_sampled(dev):
    """16,777,216 rays traced in one launch; every 16th ray compared."""
    L = synth.config_lens(3)
    rays = synth.config_rays(3)
    sel = np.arange(0, rays["x"].shape[0], 16)
    sub = {k: v[sel] for k, v in rays.items()}
    for path in [(0, 0, 0), (1, 2, 9)]:
        g = _gpu_trace(L, rays, dev, path)
        st = compare_trace(g, oracle.trace(L, sub, path, diag=True), sel=sel)
        _report(f"C3 16M {path} sampled", st)


def test_serving_lenses(dev):
    """The eight mixed lenses (4..22 surfaces, Cauchy and Sellmeier glasses)."""
    for L in synth.serve_lenses():
        rays = synth.make_rays(L, 32768, 4242)
        nr = L.n_refracting
        for path in [(0, 0, 0), (1, 1, nr), (1, nr // 2, nr // 2 + 1)]:
            st = compare_trace(_gpu_trace(L, rays, dev, path), oracle.trace(L, rays, path, diag=True))
        _report(L.name, st)


@pytest.mark.parametrize("n", [1, 63, 257, 1000])
def test_ragged_sizes(dev, n):
    L = synth.config_lens(2)
    rays = synth.make_rays(L, n, 17)
    compare_trace(_gpu_trace(L, rays, dev), oracle.trace(L, rays, diag=True))


def test_empty_launch(dev):
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    r = _to_dev(synth.make_rays(L, 4, 1), dev)
    out = lt.lt_trace(h, (0, 0, 0), r, None, n=0)
    torch.cuda.synchronize()
    assert out["x"].numel() == 0


def test_degenerate_rays(dev):
    """On-axis ray, rays pointing away from the lens, NaN and zero directions:
    no crash, the invalid ones get mask 0."""
    L = synth.config_lens(2)
    f = np.float32
    rays = {"x": np.array([0, 1, 0, np.nan, 2, 0], f), "y": np.array([0, 1, 0, 0, 1, 0], f),
            "dx": np.array([0, 0, 0, 0, 0, 0.1], f), "dy": np.array([0, 0, 0, 0, 0, 0], f),
            "dz": np.array([-1, 1, 0, -1, -1, np.nan], f),
            "lambda_nm": np.array([550, 550, 550, 550, 550, 550], f)}
    g = _gpu_trace(L, rays, dev)
    o = oracle.trace(L, rays, diag=True)
    assert g["mask"][0] == 1 and abs(g["x"][0]) < 1e-7 and abs(g["y"][0]) < 1e-7
    assert list(g["mask"][1:4]) == [0, 0, 0] and g["mask"][5] == 0
    assert g["mask"][4] == o["mask"][4]
    assert abs(g["throughput"][0] - o["throughput"][0]) < 1e-6


def test_deterministic(dev):
    L = synth.config_lens(2)
    rays = synth.make_rays(L, 100000, 9)
    a = _gpu_trace(L, rays, dev, (1, 3, 8))
    b = _gpu_trace(L, rays, dev, (1, 3, 8))
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True)


def test_plain_fp32_variant(dev):
    """The plain-FP32 option: same masks outside the boundary band; its
    exit errors are larger.  Bound: about 30 interactions x 4 FP32 roundings
    (u = 6e-8) of direction, amplified by the path's sensitivity (up to
    ~300 mm/rad in position and ~300x in direction for ghosts reflecting at
    the front surface), i.e. 2e-3 mm and 1e-4 rad."""
    L = synth.config_lens(2)
    rays = synth.config_rays(2, 262144)
    for path in [(0, 0, 0), (1, 1, 2), (1, 10, 11)]:
        st = compare_trace(_gpu_trace(L, rays, dev, path, flags=1),
                           oracle.trace(L, rays, path, diag=True), pos_tol=2e-3, ang_tol=1e-4)
        _report(f"plain FP32 {path}", st)


@pytest.mark.parametrize("cfg,path,n,flags", [(1, (0, 0, 0), 65536, 0), (2, (1, 2, 7), 100003, 0),
                                              (2, (0, 0, 0), 1, 0), (2, (1, 4, 9), 70001, 1),
                                              (3, (1, 1, 11), 1 << 20, 0)])
def test_trace_compact_matches_trace(dev, cfg, path, n, flags):
    """lt_trace_compact writes exactly the valid rays of lt_trace_ex, with
    bit-identical fields; indices are unique, and within each block of 256
    input rays they appear in input order."""
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(cfg)
    rays = synth.config_rays(cfg, n)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    r = _to_dev(rays, dev)
    full = lt.lt_trace_ex(h, path, r, None, n, flags)
    out, idx, cnt = lt.lt_trace_compact(h, path, r, flags=flags)
    torch.cuda.synchronize()
    c = int(cnt.item())
    m = full["mask"].bool()
    assert c == int(m.sum().item())
    got = idx[:c]
    order = torch.argsort(got)
    sidx = got[order]
    assert torch.equal(sidx, torch.nonzero(m).flatten())
    for k in ("x", "y", "dx", "dy", "dz", "throughput"):
        assert torch.equal(out[k][:c][order], full[k][sidx]), k
    if c == 0:
        return
    blk = (got // 256).cpu().numpy()
    g = got.cpu().numpy()
    # each block's rays are contiguous and increasing
    starts = np.flatnonzero(np.r_[True, blk[1:] != blk[:-1]])
    assert len(np.unique(blk)) == len(starts)
    same = blk[1:] == blk[:-1]
    assert np.all(g[1:][same] > g[:-1][same])
    print(f"[compact] cfg {cfg} path {path} n {n}: {c} valid", flush=True)


def test_trace_compact_empty_and_errors(dev):
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(1)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    r = _to_dev(synth.config_rays(1, 16), dev)
    cnt = torch.full((1,), -5, dtype=torch.int64, device=dev)
    lt.lt_trace_compact(h, (0, 0, 0), r, count=cnt, n=0)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    with pytest.raises(lt.LtError):
        lt.lt_trace_compact(h, (1, 2, 2), r)


@pytest.mark.parametrize("variant", ["float_pair", "fp64"])
@pytest.mark.parametrize("cfg,n", [(1, 65536), (2, 262144)])
def test_forward_tracing_all_paths(dev, cfg, n, variant):
    """LT_TRACE_FORWARD: scene-side rays from the forward input plane to the
    sensor, transmit and every two-reflection ghost, against the FP64
    oracle's forward trace (same tolerances as the sensor-side tracer), for
    the default float-pair tracer (the one the flare frame runs) and the
    FP64 variant.  Exit positions are compared for rays landing within twice
    the 36 x 24 mm frame's half-extent; grazing rays far off the sensor are
    compared in mask, direction and throughput only."""
    import paper_2605_04017_amd as lt
    L = synth.config_lens(cfg)
    rays = synth.make_forward_rays(L, n, 6000 + cfg)
    nr = L.n_refracting
    paths = [(0, 0, 0)] + [(1, j, i) for j in range(1, nr + 1) for i in range(j + 1, nr + 1)]
    if cfg == 2 and variant == "fp64":
        paths = paths[::5]
    flags = lt.LT_TRACE_FORWARD | (lt.LT_TRACE_FP64 if variant == "fp64" else 0)
    worst = 0.0
    for path in paths:
        g = _gpu_trace(L, rays, dev, path, flags=flags)
        o = oracle.trace(L, rays, path, diag=True, forward=True)
        st = compare_trace(g, o, pos_window=(2 * synth.SENSOR_HALF_W, 2 * synth.SENSOR_HALF_H))
        worst = max(worst, st.get("pos_max", 0.0))
        if path == (0, 0, 0):
            assert st["pos_compared"] > n // 20
            assert st["valid"] > n // 20
            assert np.all(g["dz"][g["mask"] == 1] > 0)
    _report(f"forward {variant} C{cfg} {len(paths)} paths", {"worst_pos": worst})


def test_forward_compact_matches(dev):
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    rays = synth.make_forward_rays(L, 50001, 77)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    r = _to_dev(rays, dev)
    full = lt.lt_trace_ex(h, (1, 2, 6), r, None, 50001, lt.LT_TRACE_FORWARD)
    out, idx, cnt = lt.lt_trace_compact(h, (1, 2, 6), r, flags=lt.LT_TRACE_FORWARD)
    torch.cuda.synchronize()
    c = int(cnt.item())
    assert c == int(full["mask"].sum().item())
    order = torch.argsort(idx[:c])
    for k in ("x", "y", "dz", "throughput"):
        assert torch.equal(out[k][:c][order], full[k][idx[:c][order]])


def _check_fp64(g, o, ulps=1.0):
    """LT_TRACE_FP64 output against the FP64 oracle: the same mask outside the
    boundary band, and every valid field within `ulps` FP32 ulps of the
    oracle's value (the FP64 result is exact to far below the FP32 rounding
    of the output)."""
    st = compare_trace(g, o, pos_tol=1e-5, ang_tol=1e-6, thr_tol=1e-5)
    both = (g["mask"] == 1) & (o["mask"] == 1)
    worst = 0.0
    for k in ("x", "y", "dx", "dy", "dz", "throughput"):
        ref = o[k][both]
        ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
        err = np.abs(g[k][both].astype(np.float64) - ref) / np.maximum(ulp, np.spacing(np.float32(1e-30)))
        assert err.max() <= ulps, (k, float(err.max()))
        worst = max(worst, float(err.max()))
    st["worst_ulps"] = worst
    return st


@pytest.mark.parametrize("cfg,n,paths", [(2, 4194304, [(0, 0, 0)]), (2, 131072, "all"), (1, 65536, "all")])
def test_fp64_variant_within_one_ulp(dev, cfg, n, paths):
    """LT_TRACE_FP64 computes in FP64: every output within one FP32 ulp of
    the FP64 oracle (the table's float-pair constants carry about 48 bits,
    far below the output rounding)."""
    import paper_2605_04017_amd as lt
    L = synth.config_lens(cfg)
    rays = synth.config_rays(cfg, n)
    nr = L.n_refracting
    if paths == "all":
        paths = [(0, 0, 0)] + [(1, j, i) for j in range(1, nr + 1) for i in range(j + 1, nr + 1)]
    worst = 0.0
    for path in paths:
        g = _gpu_trace(L, rays, dev, path, flags=lt.LT_TRACE_FP64)
        st = _check_fp64(g, oracle.trace(L, rays, path, diag=True))
        worst = max(worst, st["worst_ulps"])
    _report(f"fp64 C{cfg} {len(paths)} paths, {n} rays", {"worst_ulps": worst})


def test_fp64_variant_forward_and_flags(dev):
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    rays = synth.make_forward_rays(L, 100000, 4)
    for path in [(0, 0, 0), (1, 3, 8)]:
        g = _gpu_trace(L, rays, dev, path, flags=lt.LT_TRACE_FP64 | lt.LT_TRACE_FORWARD)
        o = oracle.trace(L, rays, path, diag=True, forward=True)
        # grazing exits far off the sensor are ill-conditioned in position
        on = (np.abs(o["x"]) <= 2 * synth.SENSOR_HALF_W) & (np.abs(o["y"]) <= 2 * synth.SENSOR_HALF_H)
        sub = lambda d: {k: (v[on] if isinstance(v, np.ndarray) and v.shape == on.shape else v)
                         for k, v in d.items()}
        _check_fp64(sub(g), sub(o), ulps=2.0)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    r = _to_dev(rays, dev)
    with pytest.raises(lt.LtError):
        lt.lt_trace_ex(h, (0, 0, 0), r, None, 100000, lt.LT_TRACE_FP64 | lt.LT_TRACE_PLAIN_FP32)
    torch.cuda.synchronize()
