"""The regressor evaluated only where the classifier says valid (Sec. 4.2,
"Neural Ray Masking"): lt_mask_index lists the set entries of a mask, and
lt_map_eval_indexed runs a one-head map on the listed rays.

lt_mask_index is checked against the mask itself (count, the set of
indices, order inside a block of 256, overflow past capacity).
lt_map_eval_indexed must reproduce, bit for bit, what lt_map_eval_ex with
LT_EVAL_GATED writes for the listed rays under an all-valid mask (the same
network; lt_map_eval is held to the oracle in test_gpu_map.py), leave the
entries past the count untouched, and the classifier -> index -> regressor
pipeline must equal the gated evaluation on the classifier's valid rays.
"""
import numpy as np
import pytest

import synth
from oracle import mlp

from test_gpu_map import gpu_map, make_params

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "dx", "dy", "dz", "throughput")


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _dev_rays(rays, dev):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in rays.items()}


@pytest.mark.parametrize("n,density,cap_frac,offset", [
    (0, 0.5, 1.0, 0), (1, 1.0, 1.0, 0), (255, 0.3, 1.0, 0), (256, 0.9, 1.0, 0), (257, 0.5, 1.0, 0),
    (16384, 1.0, 1.0, 0), (16400, 0.6, 1.0, 0), (100003, 0.17, 1.0, 0), (100003, 0.5, 0.25, 0),
    (100003, 0.3, 1.0, 5), (1 << 20, 0.02, 1.0, 0), (1 << 22, 0.166, 1.0, 3)])
def test_mask_index(dev, n, density, cap_frac, offset):
    import torch
    import paper_2605_04017_amd as lt
    rng = np.random.default_rng(n + int(100 * density))
    # set entries hold any non-zero byte; an offset start takes the unaligned path
    mask_np = np.where(rng.random(n) < density, rng.integers(1, 256, n), 0).astype(np.uint8)
    mask = torch.zeros(n + offset, dtype=torch.uint8, device=dev)[offset:]
    mask.copy_(torch.from_numpy(mask_np))
    cap = int(n * cap_frac)
    idx, cnt = lt.lt_mask_index(mask, n=n, capacity=cap)
    torch.cuda.synchronize()
    total = int(np.count_nonzero(mask_np))
    assert int(cnt.item()) == total
    k = min(total, cap)
    got = idx[:k].cpu().numpy().astype(np.int64)
    set_rays = np.nonzero(mask_np)[0]
    assert len(np.unique(got)) == k, "an index listed twice"
    assert np.all(mask_np[got] != 0), "an unset entry listed"
    if cap >= total:
        assert np.array_equal(np.sort(got), set_rays)
    # entries of one tile of 16,384 keep their order and stay together
    blk = got // 16384
    same = blk[1:] == blk[:-1]
    assert np.all(got[1:][same] > got[:-1][same])
    if cap >= total and k > 1:
        assert 1 + int((~same).sum()) == len(np.unique(blk)), "a block split into several runs"
    print(f"[mask_index] n={n} set={total} cap={cap} offset={offset}: list matches the mask", flush=True)


@pytest.mark.parametrize("width,depth,dtype,canonical,n_rays,k", [
    (32, 5, 1, 0, 50000, 7001), (32, 5, 0, 1, 30000, 4097), (32, 2, 1, 1, 9000, 1),
    (64, 3, 1, 0, 20000, 12345), (128, 5, 1, 1, 40000, 9999), (128, 5, 2, 0, 40000, 20001),
    (128, 5, 0, 0, 20000, 3001),
])
def test_eval_indexed_matches_gated(dev, width, depth, dtype, canonical, n_rays, k):
    import torch
    import paper_2605_04017_amd as lt
    rays = synth.config_rays(2, n_rays)
    desc = mlp.MapDesc(width, depth, 1, mlp.ACT_TANH, canonical=canonical)
    p = make_params(desc, 300 + width + depth + dtype, rays)
    m = gpu_map(p, dev)
    r = _dev_rays(rays, dev)
    ones = torch.ones((1, n_rays), dtype=torch.uint8, device=dev)
    ref = lt.lt_map_eval_ex(m, dtype, r, flags=lt.LT_EVAL_GATED, mask_in=ones)
    rng = np.random.default_rng(k)
    max_n = k + 500
    # an arbitrary list (any order, repeats allowed); entries past k are never evaluated
    idx_np = rng.integers(0, n_rays, max_n).astype(np.int32)
    idx = torch.from_numpy(idx_np).to(dev)
    count = torch.tensor([k], dtype=torch.int64, device=dev)
    sentinel = -12345.0
    out = {f: torch.full((1, max_n), sentinel, dtype=torch.float32, device=dev) for f in FIELDS}
    lt.lt_map_eval_indexed(m, dtype, r, idx, count, max_n, out)
    torch.cuda.synchronize()
    sel = torch.from_numpy(idx_np[:k].astype(np.int64)).to(dev)
    for f in FIELDS:
        got = out[f][0, :k].contiguous().view(torch.int32)
        want = ref[f][0][sel].contiguous().view(torch.int32)
        assert torch.equal(got, want), f"field {f} differs from the gated evaluation"
        assert bool((out[f][0, k:] == sentinel).all()), f"field {f}: an entry past the count was written"
    # no count: every one of max_n entries; a count past max_n: clamped to max_n
    for c in (None, torch.tensor([max_n + 77], dtype=torch.int64, device=dev)):
        o2 = lt.lt_map_eval_indexed(m, dtype, r, idx, c, max_n)
        torch.cuda.synchronize()
        sel2 = torch.from_numpy(idx_np.astype(np.int64)).to(dev)
        for f in FIELDS:
            assert torch.equal(o2[f][0, :max_n].contiguous().view(torch.int32),
                               ref[f][0][sel2].contiguous().view(torch.int32))
    # a zero count writes nothing
    zero = torch.zeros(1, dtype=torch.int64, device=dev)
    o3 = {f: torch.full((1, max_n), sentinel, dtype=torch.float32, device=dev) for f in FIELDS}
    lt.lt_map_eval_indexed(m, dtype, r, idx, zero, max_n, o3)
    torch.cuda.synchronize()
    for f in FIELDS:
        assert bool((o3[f] == sentinel).all())
    print(f"[indexed] {width}x{depth} dtype={dtype} canonical={canonical}: {k} listed rays bit-identical",
          flush=True)


@pytest.mark.parametrize("dtype", [1, 0])
def test_classifier_index_regressor_pipeline(dev, dtype):
    """The paper's factorised form: classifier (LT_EVAL_MASK_ONLY) ->
    lt_mask_index -> regressor on the listed rays equals the regressor under
    the classifier's mask (LT_EVAL_GATED) on every valid ray."""
    import torch
    import paper_2605_04017_amd as lt
    n = 200003
    rays = synth.config_rays(2, n)
    cls = gpu_map(make_params(mlp.MapDesc(32, 2, 1, mlp.ACT_TANH), 411, rays), dev)
    reg = gpu_map(make_params(mlp.MapDesc(32, 5, 1, mlp.ACT_TANH), 412, rays), dev)
    r = _dev_rays(rays, dev)
    cm = lt.lt_map_eval_ex(cls, dtype, r, flags=lt.LT_EVAL_MASK_ONLY)
    gated = lt.lt_map_eval_ex(reg, dtype, r, flags=lt.LT_EVAL_GATED, mask_in=cm["mask"])
    idx, cnt = lt.lt_mask_index(cm["mask"], n=n, capacity=n)
    out = lt.lt_map_eval_indexed(reg, dtype, r, idx, cnt, n)
    torch.cuda.synchronize()
    k = int(cnt.item())
    valid = cm["mask"][0].bool()
    assert k == int(valid.sum().item()) and 0 < k < n
    sel = idx[:k].long()
    assert bool(valid[sel].all())
    for f in FIELDS:
        assert torch.equal(out[f][0, :k].contiguous().view(torch.int32),
                           gated[f][0][sel].contiguous().view(torch.int32)), f"field {f}"
    print(f"[pipeline] dtype={dtype}: {k} of {n} rays valid, regressor on them alone bit-identical",
          flush=True)


def test_indexed_errors(dev):
    import ctypes as C
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd import _native as N
    rays = synth.config_rays(2, 64)
    r = _dev_rays(rays, dev)
    rs = lt._rays_struct(r, 64)
    two = gpu_map(make_params(mlp.MapDesc(32, 2, 2, mlp.ACT_TANH), 5, rays), dev)
    one = gpu_map(make_params(mlp.MapDesc(32, 2, 1, mlp.ACT_TANH), 6, rays), dev)
    buf = torch.empty(64, dtype=torch.float32, device=dev)
    idx = torch.zeros(64, dtype=torch.int32, device=dev)
    o = N.lt_map_out()
    for f in FIELDS:
        setattr(o, f, buf.data_ptr())
    call = N.lib().lt_map_eval_indexed
    assert call(two.handle, lt.LT_BF16, C.byref(rs), C.c_void_p(idx.data_ptr()), None, 64, C.byref(o), None) \
        == N.LT_ERR_ARG
    assert call(one.handle, lt.LT_BF16, C.byref(rs), None, None, 64, C.byref(o), None) == N.LT_ERR_ARG
    assert call(one.handle, lt.LT_BF16, C.byref(rs), C.c_void_p(idx.data_ptr()), None, -1, C.byref(o), None) \
        == N.LT_ERR_ARG
    assert call(one.handle, lt.LT_FP8, C.byref(rs), C.c_void_p(idx.data_ptr()), None, 64, C.byref(o), None) \
        == N.LT_ERR_DTYPE
    o.dz = None
    assert call(one.handle, lt.LT_BF16, C.byref(rs), C.c_void_p(idx.data_ptr()), None, 64, C.byref(o), None) \
        == N.LT_ERR_ARG
    assert call(one.handle, lt.LT_BF16, C.byref(rs), None, None, 0, C.byref(o), None) == N.LT_OK
    mi = N.lib().lt_mask_index
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    assert mi(None, 10, C.c_void_p(idx.data_ptr()), 10, C.c_void_p(cnt.data_ptr()), None) == N.LT_ERR_ARG
    assert mi(C.c_void_p(buf.data_ptr()), 10, None, 10, C.c_void_p(cnt.data_ptr()), None) == N.LT_ERR_ARG
    assert mi(C.c_void_p(buf.data_ptr()), 10, C.c_void_p(idx.data_ptr()), 10, None, None) == N.LT_ERR_ARG
    assert mi(C.c_void_p(buf.data_ptr()), -1, C.c_void_p(idx.data_ptr()), 10, C.c_void_p(cnt.data_ptr()), None) \
        == N.LT_ERR_ARG
    assert mi(C.c_void_p(buf.data_ptr()), 10, C.c_void_p(idx.data_ptr()), -1, C.c_void_p(cnt.data_ptr()), None) \
        == N.LT_ERR_ARG
    assert mi(None, 0, None, 0, C.c_void_p(cnt.data_ptr()), None) == N.LT_OK
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
