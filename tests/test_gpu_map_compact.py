"""Compacted map evaluation (lt_map_eval_compact; Sec. 4.2 "Neural Ray
Masking": where g(x) = 0 the map outputs nothing).

The compacted call computes the same network as lt_map_eval and must
reproduce it bit for bit: per head, count = number of set mask bits, the
bitmap equals the mask, the entries are exactly the valid rays (as a set),
and every field of every entry has the same bits as lt_map_eval's field for
that ray and head.  lt_map_eval itself is held to the oracle in
test_gpu_map.py; one test here also compares the compacted fields with the
oracle directly.  Entries of one workgroup pass (256 consecutive rays, 512
for BF16 maps narrower than 128) are contiguous and in input order.
"""
import numpy as np
import pytest

import synth
from oracle import mlp

from test_gpu_map import compare, gpu_map, make_params

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


def pass_rays(width, dtype):
    import paper_2605_04017_amd as lt
    return 512 if (dtype != lt.LT_F32 and width < 128) else 256


def check_against_full(full, c, n, P, block, cap=None, with_dz=True):
    """Every property of the compacted output against lt_map_eval's output
    (both torch tensors on the GPU)."""
    import torch
    dev = full["mask"].device
    cap = n if cap is None else cap
    shifts = torch.arange(32, device=dev, dtype=torch.int32)
    n_valid = 0
    for h in range(P):
        m = full["mask"][h]
        cnt = int(c["count"][h])
        assert cnt == int(m.sum()), f"head {h}: count {cnt} vs {int(m.sum())} valid rays"
        k = min(cnt, cap)
        n_valid += k
        idx = c["idx"][h, :k].long()
        assert bool((idx >= 0).all()) and bool((idx < n).all())
        assert bool((m[idx] == 1).all()), f"head {h}: an entry of an invalid ray"
        s = torch.sort(idx).values
        assert bool((s[1:] > s[:-1]).all()), f"head {h}: a ray written twice"
        if cap >= cnt:
            assert torch.equal(s, torch.nonzero(m).flatten()), f"head {h}: entries are not the valid rays"
        for f in FIELDS:
            if f == "dz" and not with_dz:
                continue
            got = c[f][h, :k].contiguous().view(torch.int32)
            ref = full[f][h][idx].contiguous().view(torch.int32)
            assert torch.equal(got, ref), f"head {h}: field {f} differs from lt_map_eval"
        # bitmap: bit r % 32 of word r / 32, zero past n
        if "bits" in c:
            bits = ((c["bits"][h].unsqueeze(1) >> shifts) & 1).flatten()
            assert torch.equal(bits[:n].to(torch.uint8), m), f"head {h}: bitmap differs from the mask"
            assert int(bits[n:].sum()) == 0
        # one contiguous run per workgroup pass, input order inside it
        if k > 1 and cap >= cnt:
            blk = idx // block
            same = blk[1:] == blk[:-1]
            assert bool((idx[1:][same] > idx[:-1][same]).all()), f"head {h}: order inside a pass"
            runs = 1 + int((~same).sum())
            assert runs == int(torch.unique(blk).numel()), f"head {h}: a pass split into several runs"
    return n_valid


@pytest.mark.parametrize("width,depth,heads,dtype,canonical,forward,n", [
    (128, 5, 56, 1, 1, 0, 100003),
    (128, 5, 56, 2, 1, 0, 70001),
    (128, 5, 56, 0, 1, 0, 50001),
    (128, 5, 1, 1, 0, 0, 65537),
    (128, 5, 1, 0, 0, 0, 40961),
    (128, 5, 3, 2, 0, 0, 3001),
    (64, 3, 5, 1, 0, 0, 10001),
    (64, 4, 2, 0, 0, 0, 7777),
    (32, 2, 3, 1, 1, 1, 20001),
    (32, 5, 17, 0, 0, 1, 5003),
    # the most heads a map takes: four full head blocks, every lane of the
    # reservation arrays in use
    (128, 5, 64, 1, 1, 0, 20011),
    (128, 5, 64, 2, 0, 0, 9001),
    (128, 5, 64, 0, 1, 0, 6007),
    (64, 3, 64, 1, 0, 0, 5003),
])
def test_compact_matches_eval(dev, width, depth, heads, dtype, canonical, forward, n):
    import torch
    import paper_2605_04017_amd as lt
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(width, depth, heads, mlp.ACT_TANH, canonical=canonical, forward=forward)
    p = make_params(desc, 90 + width + heads, rays)
    m = gpu_map(p, dev)
    r = _dev_rays(rays, dev)
    full = lt.lt_map_eval(m, dtype, r)
    c = lt.lt_map_eval_compact(m, dtype, r)
    torch.cuda.synchronize()
    nv = check_against_full(full, c, n, heads, pass_rays(width, dtype))
    print(f"[compact] {width}x{depth} heads={heads} dtype={dtype} n={n}: {nv} valid entries, "
          f"bit-identical to lt_map_eval", flush=True)


def test_compact_relu_and_no_dz(dev):
    """ReLU map; dz and the bitmap not requested (NULL)."""
    import torch
    import paper_2605_04017_amd as lt
    n = 30001
    rays = synth.config_rays(1, n)
    desc = mlp.MapDesc(64, 4, 4, mlp.ACT_RELU)
    p = make_params(desc, 77, rays)
    m = gpu_map(p, dev)
    r = _dev_rays(rays, dev)
    for dtype in (lt.LT_BF16, lt.LT_F32):
        full = lt.lt_map_eval(m, dtype, r)
        c = lt.lt_map_eval_compact(m, dtype, r, with_dz=False, with_bits=False)
        torch.cuda.synchronize()
        assert "dz" not in c and "bits" not in c
        check_against_full(full, c, n, 4, pass_rays(64, dtype), with_dz=False)


def test_compact_fields_against_oracle(dev):
    """The compacted fields, scattered back to their rays, against the
    oracle's BF16-emulating network (the parity test of lt_map_eval)."""
    import torch
    import paper_2605_04017_amd as lt
    n = 40000
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(128, 5, 6, mlp.ACT_TANH, canonical=1)
    p = make_params(desc, 58, rays)
    m = gpu_map(p, dev)
    c = lt.lt_map_eval_compact(m, lt.LT_BF16, _dev_rays(rays, dev))
    torch.cuda.synchronize()
    g = {"mask": np.zeros((6, n), np.uint8), "logit": np.zeros((6, n), np.float32)}
    for f in FIELDS:
        g[f] = np.full((6, n), np.nan, np.float32)
    g["throughput"][:] = 0.0
    for h in range(6):
        k = int(c["count"][h])
        idx = c["idx"][h, :k].cpu().numpy()
        g["mask"][h, idx] = 1
        for f in FIELDS:
            g[f][h, idx] = c[f][h, :k].cpu().numpy()
    # the compacted call has no logits: take the reference's, so that only
    # the mask and the fields are compared
    xhat = mlp.features(rays, p)
    ref = mlp.decode(mlp.forward_quantized(p, xhat, "bf16"), p, rays)
    g["logit"] = ref["logit"].astype(np.float32)
    compare(g, p, rays, "bf16")


@pytest.mark.parametrize("dtype", [1, 2, 0])
def test_compact_full_size_56_heads(dev, dtype):
    """The benchmarked launch: 56 heads x 16,777,216 rays of the 11-surface
    workload, compacted against uncompacted, every head and every ray."""
    import torch
    import paper_2605_04017_amd as lt
    n = 16777216
    rays = synth.config_rays(3, n)
    desc = mlp.MapDesc(128, 5, 56, mlp.ACT_TANH, canonical=1)
    p = make_params(desc, 46, {k: v[:65536] for k, v in rays.items()})
    m = gpu_map(p, dev)
    r = _dev_rays(rays, dev)
    del rays
    full = lt.lt_map_eval(m, dtype, r)
    torch.cuda.synchronize()
    cnt_max = int(full["mask"].sum(1).max())
    # capacity: the largest head's count (the benchmark's sizing)
    c = lt.lt_map_eval_compact(m, dtype, r, capacity=cnt_max)
    torch.cuda.synchronize()
    nv = check_against_full(full, c, n, 56, 256, cap=cnt_max)
    print(f"[compact full size] dtype={dtype}: {nv} valid ray-paths of {56 * n}", flush=True)
    del full, c, r
    torch.cuda.empty_cache()


def test_compact_overflow_and_empty(dev):
    import torch
    import paper_2605_04017_amd as lt
    n = 20000
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(128, 5, 3, mlp.ACT_TANH)
    p = make_params(desc, 31, rays)
    m = gpu_map(p, dev)
    r = _dev_rays(rays, dev)
    full = lt.lt_map_eval(m, lt.LT_BF16, r)
    counts = full["mask"].sum(1)
    # a capacity below the largest head's count: that head overflows
    cap = max(1, int(counts.max()) // 2)
    out = {f: torch.full((3, cap + 8), -7.0, dtype=torch.float32, device=dev) for f in FIELDS}
    out["idx"] = torch.full((3, cap + 8), -7, dtype=torch.int32, device=dev)
    out["count"] = torch.full((3,), -7, dtype=torch.int64, device=dev)
    out["bits"] = torch.empty((3, (n + 31) // 32), dtype=torch.int32, device=dev)
    c = lt.lt_map_eval_compact(m, lt.LT_BF16, r, capacity=cap, out=out)
    torch.cuda.synchronize()
    assert int(counts.max()) > cap
    # entries past the capacity stay untouched (the tensors are laid out with
    # stride cap + 8, the call with capacity cap: row h starts at h * cap)
    flat_idx = out["idx"].flatten()
    assert bool((flat_idx[3 * cap:] == -7).all())
    view = {f: out[f].flatten()[:3 * cap].view(3, cap) for f in FIELDS}
    view["idx"] = flat_idx[:3 * cap].view(3, cap)
    view["count"] = c["count"]
    view["bits"] = c["bits"]
    check_against_full(full, view, n, 3, 256, cap=cap)
    # n = 0 clears the counts and writes nothing else
    out["count"].fill_(-7)
    empty = {k: v[:0] for k, v in r.items()}
    lt.lt_map_eval_compact(m, lt.LT_BF16, empty, capacity=cap, out=out, n=0)
    torch.cuda.synchronize()
    assert out["count"].tolist() == [0, 0, 0]


def test_compact_errors(dev):
    import ctypes as C
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd import _native as N
    rays = synth.config_rays(2, 64)
    desc = mlp.MapDesc(128, 5, 2, mlp.ACT_TANH)
    p = make_params(desc, 5, rays)
    m = gpu_map(p, dev)
    r = _dev_rays(rays, dev)
    rs = lt._rays_struct(r, 64)
    buf = torch.empty(2 * 64, dtype=torch.float32, device=dev)
    idx = torch.empty(2 * 64, dtype=torch.int32, device=dev)
    cnt = torch.empty(2, dtype=torch.int64, device=dev)

    def call(n=64, cap=64, count=True, dtype=lt.LT_BF16, null_field=False):
        o = N.lt_map_compact()
        for k in FIELDS:
            setattr(o, k, buf.data_ptr())
        o.x = None if null_field else buf.data_ptr()
        o.idx = idx.data_ptr()
        o.mask_bits = None
        o.count = cnt.data_ptr() if count else None
        o.capacity = cap
        return N.lib().lt_map_eval_compact(m.handle, dtype, C.byref(rs), C.byref(o), n, None)

    assert call() == 0
    torch.cuda.synchronize()
    assert call(count=False) == N.LT_ERR_ARG
    assert call(n=-1) == N.LT_ERR_ARG
    assert call(n=1 << 31) == N.LT_ERR_ARG
    assert call(cap=-1) == N.LT_ERR_ARG
    assert call(null_field=True) == N.LT_ERR_ARG
    assert call(dtype=7) == N.LT_ERR_DTYPE
    m32 = lt.lt_map_create(32, 2, 2, lt.LT_ACT_TANH)
    o = N.lt_map_compact()
    o.count = cnt.data_ptr()
    o.capacity = 0
    assert N.lib().lt_map_eval_compact(m32.handle, lt.LT_FP8, C.byref(rs), C.byref(o), 64, None) == N.LT_ERR_DTYPE
    # parameters never set
    assert N.lib().lt_map_eval_compact(m32.handle, lt.LT_BF16, C.byref(rs), C.byref(o), 64, None) == N.LT_ERR_STATE
