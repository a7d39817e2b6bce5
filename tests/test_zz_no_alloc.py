"""lt_map_train_step_static (the training step for callers that cannot
allocate) against lt_map_train_step: two maps with the same parameters take
the same steps, one with a caller-owned workspace and one with the
library's static scratch.  Both run the same deterministic kernels on the
same inputs, so losses, parameters and Adam moments must agree bit for bit:
first at the largest batch the scratch holds, then with a smaller, ragged
batch in a row (the scratch keeps the previous call's content)."""
import numpy as np
import pytest

import synth
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _params(desc, seed, rays):
    p = mlp.init_params(desc, seed)
    x = np.stack([rays[k].astype(np.float64) for k in synth.RAY_FIELDS], 1)
    p.in_shift = x.mean(0).astype(np.float32).astype(np.float64)
    p.in_scale = (1.0 / x.std(0)).astype(np.float32).astype(np.float64)
    return p


def _map(p, dev):
    import torch
    import paper_2605_04017_amd as lt
    d = p.desc
    m = lt.lt_map_create(d.width, d.depth, d.n_heads, d.activation)
    lt.lt_map_set_params(m, torch.from_numpy(p.flat().astype(np.float32)).to(dev))
    lt.lt_map_set_norm(m, p.in_shift, p.in_scale, p.out_shift.reshape(-1), p.out_scale.reshape(-1))
    return m


def _largest_batch(lt, m):
    """Largest n whose workspace fits the static scratch (bisection on the
    library's own size function)."""
    lo, hi = 1, 1 << 22
    assert lt.lt_map_workspace_bytes(m, lo) <= lt.LT_STATIC_SCRATCH_BYTES
    assert lt.lt_map_workspace_bytes(m, hi) > lt.LT_STATIC_SCRATCH_BYTES
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if lt.lt_map_workspace_bytes(m, mid) <= lt.LT_STATIC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("width,depth", [(128, 5), (32, 2)])
def test_static_scratch_step_matches_workspace_step(dev, width, depth):
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    desc = mlp.MapDesc(width, depth, 1, mlp.ACT_TANH)
    probe = _params(desc, 61, synth.config_rays(2, 4096))
    a, b = _map(probe, dev), _map(probe, dev)
    n1 = min(_largest_batch(lt, a), 1 << 20)
    n2 = n1 // 3 + 17
    print(f"[no-alloc] {width} x {depth}: batches {n1} then {n2}", flush=True)
    rays_np = synth.config_rays(2, n1 + n2)
    rays = {k: torch.from_numpy(v).to(dev) for k, v in rays_np.items()}
    ex = lt.lt_trace(h, (0, 0, 0), rays)
    for k, (lo, n) in enumerate(((0, n1), (n1, n2)), 1):
        rb = {f: v[lo:lo + n] for f, v in rays.items()}
        tb = {"valid": ex["mask"][lo:lo + n].reshape(1, -1)}
        for f in ("x", "y", "dx", "dy", "throughput"):
            tb[f] = ex[f][lo:lo + n].reshape(1, -1)
        cfg = {"lr": 1e-3, "step": k, "w_bce": 1.0, "w_l2": 2.0}
        ws = lt.workspace(a, n)
        la = lt.lt_map_train_step(a, rb, tb, cfg, ws)
        lb = lt.lt_map_train_step_static(b, rb, tb, cfg)
        torch.cuda.synchronize()
        del ws
        assert torch.equal(la, lb), f"step {k}: loss {la.tolist()} vs {lb.tolist()}"
        assert torch.equal(lt.lt_map_get_params(a), lt.lt_map_get_params(b)), f"step {k}: parameters"
        assert torch.equal(lt.lt_map_adam_state(a), lt.lt_map_adam_state(b)), f"step {k}: moments"
        assert float(la[0]) > 0.0


def test_static_scratch_rejects_oversized_batch(dev):
    """A batch beyond the scratch is refused before anything is enqueued."""
    import torch
    import paper_2605_04017_amd as lt
    desc = mlp.MapDesc(128, 5, 1, mlp.ACT_TANH)
    rays_np = synth.config_rays(2, 4096)
    m = _map(_params(desc, 62, rays_np), dev)
    n = 1 << 15
    assert lt.lt_map_workspace_bytes(m, n) > lt.LT_STATIC_SCRATCH_BYTES
    rays = {k: torch.zeros(n, dtype=torch.float32, device=dev) for k in synth.RAY_FIELDS}
    t = {"valid": torch.zeros((1, n), dtype=torch.uint8, device=dev)}
    for f in ("x", "y", "dx", "dy", "throughput"):
        t[f] = torch.zeros((1, n), dtype=torch.float32, device=dev)
    before = lt.lt_map_get_params(m).clone()
    with pytest.raises(lt.LtError) as e:
        lt.lt_map_train_step_static(m, rays, t, {"lr": 1e-3, "step": 1})
    assert e.value.status == lt.LT_ERR_ARG and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(before, lt.lt_map_get_params(m))
