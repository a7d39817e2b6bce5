"""Serving on the GPU: continuous batching over HIP streams for eight
resident lenses and maps; every request's result equals the result of the
same request run alone (the kernels are per-ray independent)."""
import numpy as np
import pytest

import synth
from oracle import mlp

pytestmark = pytest.mark.gpu


def _setup(dev, mode):
    import torch
    import paper_2605_04017_amd as lt
    lenses = synth.serve_lenses()
    hl, maps, pools = [], [], []
    for i, L in enumerate(lenses):
        hl.append(lt.lt_lens_create(L.surfaces, L.glasses))
        rays = synth.make_rays(L, 200000, 5000 + i)
        pools.append({k: torch.from_numpy(v).to(dev) for k, v in rays.items()})
        p = mlp.init_params(mlp.MapDesc(128, 5, 1), 60 + i)
        m = lt.lt_map_create(128, 5, 1)
        lt.lt_map_set_params(m, torch.from_numpy(p.flat().astype(np.float32)).to(dev))
        maps.append(m)
    return hl, maps, pools


@pytest.mark.parametrize("mode,dtype", [("map", 1), ("map", 0), ("trace", 0)])
def test_mixed_equals_alone(mode, dtype):
    import torch
    from paper_2605_04017_amd.serve import GpuExecutor, Scheduler, latency_stats, poisson_requests, run_trace
    dev = torch.device("cuda:0")
    hl, maps, pools = _setup(dev, mode)
    reqs = poisson_requests(60, 4000.0, 8, seed=77, min_rays=1000, max_rays=150000)
    for r in reqs:
        off = (r.rid * 7919) % (200000 - r.n)
        r.payload = {k: v[off:off + r.n] for k, v in pools[r.lens].items()}
    outs = {r.rid: [] for r in reqs}
    ex = GpuExecutor(4, hl, maps, mode, dtype, outs)
    sched = Scheduler(ex, mem_budget_bytes=2 << 30, bytes_per_ray=64, chunk=65536)
    ex.start_clock()
    done = run_trace(sched, reqs, ex.clock)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    st = latency_stats(done)
    print(f"[serve {mode} dtype {dtype}] p50 {st['p50_ms']:.3f} ms p99 {st['p99_ms']:.3f} ms", flush=True)
    import paper_2605_04017_amd as lt
    for r in reqs[::5]:
        if mode == "map":
            alone = lt.lt_map_eval(maps[r.lens], dtype, r.payload)
        else:
            alone = lt.lt_trace(hl[r.lens], (0, 0, 0), r.payload)
        torch.cuda.synchronize()
        for lo, hi, o in outs[r.rid]:
            for k in alone:
                a = alone[k][..., lo:hi]
                b = o[k]
                assert torch.equal(torch.nan_to_num(a.float(), nan=-7.0),
                                   torch.nan_to_num(b.float(), nan=-7.0)), (r.rid, k)


def _payloads(reqs, pools, mode, n_heads=1):
    import paper_2605_04017_amd as lt
    for r in reqs:
        off = (r.rid * 7919) % (200000 - r.n + 1)
        rays = {k: v[off:off + r.n] for k, v in pools[r.lens].items()}
        dev = rays["x"].device
        out = lt.empty_map_out(n_heads, r.n, dev) if mode == "map" else lt.empty_exit(r.n, dev)
        r.payload = (rays, out)


def _same(a, b):
    import torch
    return torch.equal(torch.nan_to_num(a.float(), nan=-7.0), torch.nan_to_num(b.float(), nan=-7.0))


@pytest.mark.parametrize("mode,dtype", [("map", 1), ("map", 2), ("map", 0), ("trace", 0)])
def test_native_mixed_equals_alone(mode, dtype):
    """The native loop (lt_server_*): every request, chunked and interleaved
    with others on four streams, gives bit for bit the result of the same
    request evaluated alone; edge sizes (empty, one ray, exactly one chunk,
    one ray past a chunk) included."""
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd.serve import NativeScheduler, Request, latency_stats, poisson_requests, run_trace
    dev = torch.device("cuda:0")
    hl, maps, pools = _setup(dev, mode)
    if mode == "map":
        for m in maps:
            lt.lt_map_quantize(m, dtype)
    reqs = poisson_requests(60, 4000.0, 8, seed=78, min_rays=1000, max_rays=150000)
    t_last = reqs[-1].arrival
    for i, n in enumerate((0, 1, 16384, 16385)):
        reqs.append(Request(len(reqs), i % 8, n, t_last + 1e-4 * i))
    _payloads(reqs, pools, mode)
    torch.cuda.synchronize()
    srv = lt.Server(4, chunk=16384, mem_budget=2 << 30, bytes_per_ray=64)
    sched = NativeScheduler(srv, hl, maps, mode, dtype)
    done = run_trace(sched, reqs, sched.clock)
    torch.cuda.synchronize()
    assert len(done) == len(reqs) and not sched.rejected
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert all(r.done >= 0.0 for r in done)
    _, launches = srv.stats()
    assert launches == sum(-(-r.n // 16384) for r in reqs)
    st = latency_stats(done)
    print(f"[native serve {mode} dtype {dtype}] {len(done)} requests, {launches} launches, "
          f"p50 {st['p50_ms']:.3f} ms p99 {st['p99_ms']:.3f} ms", flush=True)
    for r in reqs:
        rays, out = r.payload
        if mode == "map":
            alone = lt.lt_map_eval(maps[r.lens], dtype, rays, None, r.n)
        else:
            alone = lt.lt_trace(hl[r.lens], (0, 0, 0), rays, None, r.n)
        torch.cuda.synchronize()
        for k in alone:
            assert _same(alone[k], out[k]), (r.rid, r.n, k)
    srv.close()


def test_native_budget_admission_and_rejection():
    """Admission by memory: the accounted in-flight bytes never exceed the
    budget, a request larger than the whole budget is refused at submission
    (LT_ERR_ARG) and the others all complete."""
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd.serve import NativeScheduler, poisson_requests, run_trace
    dev = torch.device("cuda:0")
    hl, maps, pools = _setup(dev, "trace")
    reqs = poisson_requests(40, 1e9, 8, seed=79, min_rays=1000, max_rays=120000)
    budget = 150000 * 64
    _payloads(reqs, pools, "trace")
    srv = lt.Server(3, chunk=32768, mem_budget=budget, bytes_per_ray=64)
    sched = NativeScheduler(srv, hl, maps, "trace")
    done = run_trace(sched, reqs, sched.clock)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    max_in_use, _ = srv.stats()
    assert 0 < max_in_use <= budget
    big = {k: v[:150001] for k, v in pools[0].items()}
    with pytest.raises(lt.LtError) as e:
        srv.submit_trace(hl[0], (0, 0, 0), big, lt.empty_exit(150001, dev), 150001, 999)
    assert e.value.status == lt.LT_ERR_ARG
    print(f"[native serve] budget {budget} B, largest in flight {max_in_use} B", flush=True)
    srv.close()


def test_native_multi_head_map_and_stale_weights():
    """A three-head map keeps its head-major output layout (its requests run
    whole, whatever the chunk), and submitting against packed weights that
    are older than the parameters is refused (LT_ERR_STATE)."""
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd.serve import NativeScheduler, Request, run_trace
    dev = torch.device("cuda:0")
    L = synth.serve_lenses()[0]
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    pool = {k: torch.from_numpy(v).to(dev) for k, v in synth.make_rays(L, 200000, 5100).items()}
    p = mlp.init_params(mlp.MapDesc(128, 5, 3), 61)
    m = lt.lt_map_create(128, 5, 3)
    lt.lt_map_set_params(m, torch.from_numpy(p.flat().astype(np.float32)).to(dev))
    lt.lt_map_quantize(m, lt.LT_BF16)
    reqs = [Request(i, 0, n, 0.0) for i, n in enumerate((70000, 5000, 40000))]
    _payloads(reqs, [pool], "map", n_heads=3)
    srv = lt.Server(2, chunk=8192, mem_budget=1 << 30, bytes_per_ray=64)
    sched = NativeScheduler(srv, [h], [m], "map", lt.LT_BF16)
    run_trace(sched, reqs, sched.clock)
    torch.cuda.synchronize()
    assert srv.stats()[1] == len(reqs)
    for r in reqs:
        rays, out = r.payload
        alone = lt.lt_map_eval(m, lt.LT_BF16, rays, None, r.n)
        torch.cuda.synchronize()
        for k in alone:
            assert _same(alone[k], out[k]), (r.rid, k)
    lt.lt_map_set_params(m, torch.from_numpy(p.flat().astype(np.float32)).to(dev))
    rays, out = reqs[1].payload
    with pytest.raises(lt.LtError) as e:
        srv.submit_map(m, lt.LT_BF16, rays, out, reqs[1].n, 7)
    assert e.value.status == lt.LT_ERR_STATE
    srv.close()


def test_native_submit_rejects_missing_fields():
    """Submission checks ray and output pointers on the host (LT_ERR_ARG),
    so a bad request never reaches a launch."""
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd import _native as N
    import ctypes as C
    dev = torch.device("cuda:0")
    L = synth.serve_lenses()[0]
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    srv = lt.Server(1, chunk=1024, mem_budget=1 << 20, bytes_per_ray=1)
    rays, ex, p = N.lt_rays(), N.lt_exit(), N.lt_path(0, 0, 0)
    st = N.lib().lt_server_submit_trace(srv.handle, h.handle, C.byref(p), C.byref(rays), C.byref(ex), 16, 1)
    assert st == N.LT_ERR_ARG
    assert N.lib().lt_server_submit_trace(srv.handle, h.handle, C.byref(p), C.byref(rays), C.byref(ex), 0,
                                          2) == N.LT_OK
    done, n_open = srv.poll()
    assert [d[0] for d in done] == [2] and n_open == 0
    srv.close()
    torch.cuda.synchronize()
