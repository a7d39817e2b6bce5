"""GPU training path: hand-written backward (lt_map_backward), fused train
step (loss + backward + Adam), autograd.Function, checkpoint/resume, and a
fit on rays the GPU tracer generates.

Gradient parity is against the FP64 reference with the kernels' BF16
rounding (oracle/mlp.py: forward_quantized_cache + backward_quantized).  As
in the forward tests, FP32 summation-order differences occasionally move a
BF16-rounded activation or gradient by one BF16 ulp, so layer gradients are
compared in relative Frobenius norm (bound 2e-2; BF16 unit roundoff is
3.9e-3) rather than element by element.
"""
import numpy as np
import pytest

import synth
from oracle import mlp

pytestmark = pytest.mark.gpu

GRAD_TOL = 2e-2


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def make_params(desc, seed, rays):
    p = mlp.init_params(desc, seed)
    rng = np.random.default_rng(seed)
    for b in p.b:
        b[:] = rng.normal(0, 0.2, b.shape)
    x = np.stack([rays[k].astype(np.float64) for k in synth.RAY_FIELDS], 1)
    p.in_shift = x.mean(0).astype(np.float32).astype(np.float64)
    sd = x.std(0)
    sd[sd == 0] = 1.0   # the y slot of canonical inputs is always 0
    p.in_scale = (1.0 / sd).astype(np.float32).astype(np.float64)
    H = desc.n_heads
    p.out_shift = rng.normal(0, 1, (H, 5)).astype(np.float32).astype(np.float64)
    p.out_scale = rng.uniform(0.5, 2.0, (H, 5)).astype(np.float32).astype(np.float64)
    p.set_flat(p.flat().astype(np.float32).astype(np.float64))
    return p


def gpu_map(p, dev):
    import torch
    import paper_2605_04017_amd as lt
    d = p.desc
    m = lt.lt_map_create(d.width, d.depth, d.n_heads, d.activation, d.canonical)
    lt.lt_map_set_params(m, torch.from_numpy(p.flat().astype(np.float32)).to(dev))
    lt.lt_map_set_norm(m, p.in_shift, p.in_scale, p.out_shift.reshape(-1), p.out_scale.reshape(-1))
    return m


def to_dev(rays, dev):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in rays.items()}


def split_layers(p, flat):
    q = p.copy()
    q.set_flat(flat.astype(np.float64))
    return list(zip(q.W, q.b))


def compare_grads(p, g_gpu, g_ref, tol=GRAD_TOL):
    worst = 0.0
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(split_layers(p, g_gpu), g_ref)):
        for a, r, what in ((gW, rW, "W"), (gb, rb, "b")):
            e = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
            worst = max(worst, e)
            assert e <= tol, f"layer {li} {what}: relative gradient error {e:.3e}"
    return worst


@pytest.mark.parametrize("width,depth,heads,act,n", [(64, 3, 2, 0, 3000), (128, 5, 1, 0, 20000),
                                                      (64, 4, 1, 1, 5000), (128, 5, 56, 0, 2048),
                                                      (32, 2, 3, 0, 77), (128, 3, 9, 0, 4097),
                                                      (64, 2, 5, 0, 999)])
def test_backward_matches_reference(dev, width, depth, heads, act, n):
    import torch
    import paper_2605_04017_amd as lt
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(width, depth, heads, act)
    p = make_params(desc, 100 + width + heads, rays)
    m = gpu_map(p, dev)
    r = to_dev(rays, dev)
    o, ws = lt.lt_map_forward_train(m, r)
    rng = np.random.default_rng(5)
    d_out = rng.normal(0, 1e-3, (6 * heads, n)).astype(np.float32)
    g = lt.lt_map_backward(m, torch.from_numpy(d_out).to(dev), ws)
    torch.cuda.synchronize()
    o_ref, cache = mlp.forward_quantized_cache(p, mlp.features(rays, p))
    eo = np.abs(o.cpu().numpy().T - o_ref)
    assert np.median(eo) < 1e-5 and np.quantile(eo, 0.99) < 2e-3 and eo.max() < 2e-2
    g_ref = mlp.backward_quantized(p, cache, d_out.T.astype(np.float64))
    worst = compare_grads(p, g.cpu().numpy(), g_ref)
    print(f"[grad parity] {desc} n={n}: worst relative layer error {worst:.2e}", flush=True)


def test_gradient_against_finite_differences(dev):
    """GPU gradient of the loss vs central differences of the FP64 loss, on
    the largest-magnitude components."""
    import torch
    import paper_2605_04017_amd as lt
    n = 4000
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(32, 3, 1, mlp.ACT_TANH)
    p = make_params(desc, 7, rays)
    rng = np.random.default_rng(8)
    valid = rng.integers(0, 2, (1, n))
    tnorm = rng.normal(0, 1, (1, n, 5))
    xhat = mlp.features(rays, p)
    m = gpu_map(p, dev)
    r = to_dev(rays, dev)
    o, ws = lt.lt_map_forward_train(m, r)
    # gradient of the loss with respect to the GPU's own outputs
    _, d_out = mlp.loss_terms(p, o.cpu().numpy().T.astype(np.float64), valid, tnorm)
    g = lt.lt_map_backward(m, torch.from_numpy(d_out.T.astype(np.float32)).contiguous().to(dev), ws)
    g = g.cpu().numpy().astype(np.float64)
    theta = p.flat()
    idx = np.argsort(-np.abs(g))[:25]
    for k in idx:
        h = 1e-4 * max(1.0, abs(theta[k]))
        q = p.copy()
        th = theta.copy()
        th[k] += h
        q.set_flat(th)
        lp = mlp.loss_and_grad(q, xhat, valid, tnorm)[0][0]
        th[k] -= 2 * h
        q.set_flat(th)
        lm = mlp.loss_and_grad(q, xhat, valid, tnorm)[0][0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 3e-2 * abs(fd) + 1e-6, (k, fd, g[k])


def _targets(lens, rays_np, dev, nheads=1):
    """Traced targets (GPU tracer) for the transmit path."""
    import torch
    import paper_2605_04017_amd as lt
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    r = to_dev(rays_np, dev)
    ex = lt.lt_trace(h, (0, 0, 0), r)
    t = {"valid": ex["mask"].reshape(1, -1).contiguous()}
    for k in ("x", "y", "dx", "dy", "throughput"):
        t[k] = ex[k].reshape(1, -1).contiguous()
    return r, t


def test_train_step_loss_and_update(dev):
    """Loss of the fused step equals the reference loss of the same forward;
    the Adam update moves parameters by the reference step where the
    reference gradient is well above rounding noise."""
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    n = 16384
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(64, 3, 1, mlp.ACT_TANH)
    p = make_params(desc, 9, rays)
    m = gpu_map(p, dev)
    r, t = _targets(L, rays, dev)
    ws = lt.workspace(m, n)
    cfg = {"lr": 1e-3, "beta1": 0.9, "beta2": 0.999, "eps": 1e-8, "step": 1, "w_bce": 1.0, "w_l2": 1.0}
    loss = lt.lt_map_train_step(m, r, t, cfg, ws)
    torch.cuda.synchronize()
    tn = {k: v.cpu().numpy() for k, v in t.items()}
    valid = tn["valid"].astype(np.int64)
    tnorm = np.stack([tn[k][0] for k in ("x", "y", "dx", "dy", "throughput")], -1)[None]
    tnorm = (tnorm - p.out_shift[:, None, :]) / p.out_scale[:, None, :]
    (lref, bref, l2ref), gref = mlp.loss_and_grad_quantized(p, mlp.features(rays, p), valid, tnorm)
    lg = loss.cpu().numpy()
    assert abs(lg[0] - lref) <= 1e-3 * lref and abs(lg[1] - bref) <= 1e-3 * bref
    new = lt.lt_map_get_params(m).cpu().numpy().astype(np.float64)
    step = new - p.flat()
    gr = mlp.grads_flat(gref)
    big = np.abs(gr) > 1e-2 * np.abs(gr).max()
    # first Adam step: -lr * g / (|g| + eps)
    expect = -1e-3 * gr / (np.abs(gr) + 1e-8)
    assert np.mean(np.abs(step[big] - expect[big]) < 1e-6) > 0.99


def test_training_reduces_loss_and_resumes_exactly(dev):
    """Fit the map on GPU-traced rays; checkpoint/resume is bit-exact."""
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    n = 65536
    rays = synth.config_rays(2, n)
    r, t = _targets(L, rays, dev)
    desc = mlp.MapDesc(64, 3, 1, mlp.ACT_TANH)
    p = make_params(desc, 11, rays)
    tv = {k: v.cpu().numpy()[0] for k, v in t.items()}
    ok = tv["valid"] == 1
    reg = np.stack([tv[k][ok] for k in ("x", "y", "dx", "dy", "throughput")], 1)
    p.out_shift = reg.mean(0)[None].astype(np.float32).astype(np.float64)
    p.out_scale = reg.std(0)[None].astype(np.float32).astype(np.float64)
    params0 = torch.from_numpy(p.flat().astype(np.float32)).to(dev)

    def run(m, steps, start=1):
        ws = lt.workspace(m, n)
        losses = []
        for k in range(start, start + steps):
            cfg = {"lr": 3e-3, "step": k}
            losses.append(float(lt.lt_map_train_step(m, r, t, cfg, ws).cpu()[0]))
        return losses

    a = gpu_map(p, dev)
    la = run(a, 60)
    assert la[-1] < 0.5 * la[0], (la[0], la[-1])
    # 60 straight == 25 + save/restore into a fresh map + 35
    b = gpu_map(p, dev)
    lt.lt_map_set_params(b, params0)
    run(b, 25)
    theta = lt.lt_map_get_params(b).clone()
    mv = lt.lt_map_adam_state(b).clone()
    c = gpu_map(p, dev)
    lt.lt_map_set_params(c, theta)
    lt.lt_map_adam_state(c, mv, to_map=True)
    run(c, 35, start=26)
    torch.cuda.synchronize()
    assert torch.equal(lt.lt_map_get_params(a), lt.lt_map_get_params(c))
    print(f"[train] loss {la[0]:.4f} -> {la[-1]:.4f} in 60 steps", flush=True)


def test_autograd_function(dev):
    """torch.autograd through the hand-written kernels equals lt_map_backward."""
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd.autograd import map_forward
    n = 5000
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(64, 3, 2, mlp.ACT_TANH)
    p = make_params(desc, 13, rays)
    m = gpu_map(p, dev)
    r = to_dev(rays, dev)
    params = torch.from_numpy(p.flat().astype(np.float32)).to(dev).requires_grad_(True)
    o = map_forward(params, r, m)
    w = torch.randn_like(o) * 1e-3
    (o * w).sum().backward()
    o2, ws = lt.lt_map_forward_train(m, r)
    g2 = lt.lt_map_backward(m, w.contiguous(), ws)
    assert torch.equal(o.detach(), o2)
    assert torch.equal(params.grad, g2)


def test_canonical_train_step(dev):
    """Canonical-input map: the fused step moves the traced targets into
    each ray's canonical frame; loss and first Adam step match the reference
    (oracle normalise_targets with the rays)."""
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    n = 16384
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(64, 3, 1, mlp.ACT_TANH, canonical=True)
    p = make_params(desc, 29, mlp.canonical_frame(rays)[0])
    m = gpu_map(p, dev)
    r, t = _targets(L, rays, dev)
    ws = lt.workspace(m, n)
    cfg = {"lr": 1e-3, "step": 1, "w_bce": 1.0, "w_l2": 1.0}
    loss = lt.lt_map_train_step(m, r, t, cfg, ws)
    torch.cuda.synchronize()
    tn = {k: v.cpu().numpy() for k, v in t.items()}
    valid = tn["valid"].astype(np.int64)
    tnorm = mlp.normalise_targets({k: tn[k] for k in ("x", "y", "dx", "dy", "throughput")}, p, rays)
    (lref, bref, l2ref), gref = mlp.loss_and_grad_quantized(p, mlp.features(rays, p), valid, tnorm)
    lg = loss.cpu().numpy()
    assert abs(lg[0] - lref) <= 1e-3 * lref and abs(lg[2] - l2ref) <= 2e-3 * l2ref
    new = lt.lt_map_get_params(m).cpu().numpy().astype(np.float64)
    step = new - p.flat()
    gr = mlp.grads_flat(gref)
    big = np.abs(gr) > 1e-2 * np.abs(gr).max()
    expect = -1e-3 * gr / (np.abs(gr) + 1e-8)
    assert np.mean(np.abs(step[big] - expect[big]) < 1e-6) > 0.99


def test_cosine_direction_loss_train_step(dev):
    """w_cos > 0: squared error on x, y, throughput plus 1 - cos of the exit
    direction; the fused step's loss and first Adam step match the
    reference (loss_and_grad_quantized with w_cos)."""
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    n = 16384
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(64, 3, 1, mlp.ACT_TANH)
    p = make_params(desc, 37, rays)
    r, t = _targets(L, rays, dev)
    tv = {k: v.cpu().numpy()[0] for k, v in t.items()}
    ok = tv["valid"] == 1
    reg = np.stack([tv[k][ok] for k in ("x", "y", "dx", "dy", "throughput")], 1)
    p.out_shift = reg.mean(0)[None].astype(np.float32).astype(np.float64)
    p.out_scale = reg.std(0)[None].astype(np.float32).astype(np.float64)
    m = gpu_map(p, dev)
    ws = lt.workspace(m, n)
    cfg = {"lr": 1e-3, "step": 1, "w_bce": 0.5, "w_l2": 1.0, "w_cos": 20.0}
    loss = lt.lt_map_train_step(m, r, t, cfg, ws)
    torch.cuda.synchronize()
    tn = {k: v.cpu().numpy() for k, v in t.items()}
    tnorm = mlp.normalise_targets({k: tn[k] for k in ("x", "y", "dx", "dy", "throughput")}, p)
    (lref, bref, rref), gref = mlp.loss_and_grad_quantized(p, mlp.features(rays, p),
                                                           tn["valid"].astype(np.int64), tnorm,
                                                           0.5, 1.0, 20.0)
    lg = loss.cpu().numpy()
    assert abs(lg[0] - lref) <= 1e-3 * lref and abs(lg[2] - rref) <= 2e-3 * rref, (lg, lref, rref)
    new = lt.lt_map_get_params(m).cpu().numpy().astype(np.float64)
    step = new - p.flat()
    gr = mlp.grads_flat(gref)
    big = np.abs(gr) > 1e-2 * np.abs(gr).max()
    expect = -1e-3 * gr / (np.abs(gr) + 1e-8)
    assert np.mean(np.abs(step[big] - expect[big]) < 1e-6) > 0.99
    with pytest.raises(lt.LtError):
        lt.lt_map_train_step(m, r, t, {"lr": 1e-3, "step": 2, "w_cos": -1.0}, ws)


# ------------------------------------------- element-wise step parity ----

def _trace_targets(lens, rays_np, dev, heads):
    """Traced targets of the first `heads` paths (transmit, then the ghosts
    in lt_ghost_index order) from the GPU tracer, head-major [heads][n]."""
    import torch
    import paper_2605_04017_amd as lt
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    r = to_dev(rays_np, dev)
    nr = lens.n_refracting
    paths = [(0, 0, 0)] + [(1, j, i) for j in range(1, nr + 1) for i in range(j + 1, nr + 1)]
    n = rays_np["x"].shape[0]
    t = {"valid": torch.empty((heads, n), dtype=torch.uint8, device=dev)}
    for k in ("x", "y", "dx", "dy", "throughput"):
        t[k] = torch.empty((heads, n), dtype=torch.float32, device=dev)
    for p_i, path in enumerate(paths[:heads]):
        ex = lt.lt_trace(h, path, r)
        t["valid"][p_i] = ex["mask"]
        for k in ("x", "y", "dx", "dy", "throughput"):
            t[k][p_i] = ex[k]
    torch.cuda.synchronize()
    return r, t


def _fit_norm(p, t):
    """Per-head output normalisation from the valid traced targets."""
    tv = {k: v.cpu().numpy() for k, v in t.items()}
    for hd in range(p.desc.n_heads):
        ok = tv["valid"][hd] == 1
        if ok.sum() < 2:
            continue
        reg = np.stack([tv[k][hd][ok] for k in ("x", "y", "dx", "dy", "throughput")], 1)
        sd = reg.std(0)
        sd[sd == 0] = 1.0
        p.out_shift[hd] = reg.mean(0).astype(np.float32)
        p.out_scale[hd] = sd.astype(np.float32)
    return tv


# Element-wise bound of a GPU gradient g against the reference g_ref of one
# layer: |g - g_ref| <= GRAD_A |g_ref| + GRAD_B max|g_ref|.  Every gradient
# element is a sum over the batch; the two sides differ by FP32 accumulation
# (relative ~ sqrt(K) 2^-24 per product sum, far below GRAD_A) and by the
# BF16 roundings that FP32 noise moves across a rounding boundary.  Such a
# flip changes one rounded activation or hidden gradient by one BF16 ulp
# (2^-8 of it); it hits a fraction f of the batch's terms (f ~ FP32 error /
# BF16 ulp ~ 1e-3) with random sign, so it moves an element by about
# 2^-8 sqrt(f n) |term|, while the largest element of a layer is a coherent
# sum of ~0.1 n |term|: at n = 65,536 the ratio is ~1e-5, and GRAD_B = 1e-4
# leaves a factor of ten.
GRAD_A, GRAD_B = 2.0 ** -8, 1e-4


def _elementwise(p, g_gpu, g_ref, what):
    worst = 0.0
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(split_layers(p, g_gpu), g_ref)):
        for a, r, nm in ((gW, rW, "W"), (gb, rb, "b")):
            scale = np.abs(r).max()
            bound = GRAD_A * np.abs(r) + GRAD_B * scale
            ex = np.abs(a - r) / np.maximum(bound, 1e-300)
            worst = max(worst, float(ex.max()))
            assert np.all(np.abs(a - r) <= bound), (
                f"{what} layer {li} {nm}: {int((np.abs(a - r) > bound).sum())} of {r.size} elements "
                f"outside the bound, worst |g - g_ref| / max|g_ref| = "
                f"{float(np.abs(a - r).max() / scale):.3e}")
    return worst


@pytest.mark.parametrize("width,depth,heads,n,steps", [(128, 5, 1, 65536, 10), (128, 5, 56, 65536, 4),
                                                       (64, 3, 1, 16384, 3)])
def test_train_step_elementwise(dev, width, depth, heads, n, steps):
    """The fused lt_map_train_step at the training configuration's shape
    (5 x 128 trunk, batch 65,536; one head and the 56-path map) over several
    Adam steps.  Per step: the loss components against the reference loss
    of the same parameters (1e-3 relative); the step's gradient, read back
    from the Adam moments as g = (m_new - beta1 m_old) / (1 - beta1), element
    by element against the reference gradient with the kernels' BF16
    rounding; and the second moment and the parameters against the oracle's
    Adam step driven by that gradient."""
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    rays = synth.config_rays(2, n)
    desc = mlp.MapDesc(width, depth, heads, mlp.ACT_TANH)
    p = make_params(desc, 300 + heads, rays)
    r, t = _trace_targets(L, rays, dev, heads)
    tv = _fit_norm(p, t)
    m = gpu_map(p, dev)
    ws = lt.workspace(m, n)
    valid = tv["valid"].astype(np.int64)
    tnorm = mlp.normalise_targets({k: tv[k] for k in ("x", "y", "dx", "dy", "throughput")}, p)
    # the ABI passes the optimiser settings as FP32 (lt_train_cfg), so the
    # reference step runs on exactly those values: 1 - beta2 differs from
    # 1e-3 by 1.3e-5 relative in FP32
    b1, b2, eps, lr = (float(np.float32(v)) for v in (0.9, 0.999, 1e-8, 2e-3))
    P = m.n_params
    theta = lt.lt_map_get_params(m).cpu().numpy().astype(np.float64)
    mv = np.zeros(2 * P)
    worst = 0.0
    for k in range(1, steps + 1):
        cfg = {"lr": lr, "beta1": b1, "beta2": b2, "eps": eps, "step": k, "w_bce": 1.0, "w_l2": 1.0}
        loss = lt.lt_map_train_step(m, r, t, cfg, ws).cpu().numpy().astype(np.float64)
        theta_new = lt.lt_map_get_params(m).cpu().numpy().astype(np.float64)
        mv_new = lt.lt_map_adam_state(m).cpu().numpy().astype(np.float64).reshape(-1)
        q = p.copy()
        q.set_flat(theta)
        (lref, bref, l2ref), gref = mlp.loss_and_grad_quantized(q, mlp.features(rays, q), valid, tnorm)
        for got, ref, nm in ((loss[0], lref, "total"), (loss[1], bref, "bce"), (loss[2], l2ref, "l2")):
            assert abs(got - ref) <= 1e-3 * abs(ref), f"step {k} {nm} loss {got} vs {ref}"
        g = (mv_new[:P] - b1 * mv[:P]) / (1.0 - b1)
        worst = max(worst, _elementwise(q, g, gref, f"step {k}"))
        st = mlp.AdamState(mv[:P].copy(), mv[P:].copy(), k - 1)
        mlp.adam_step(q, g, st, lr, b1, b2, eps)
        # FP32 on the device: v to a few ulps; the update to a few ulps of
        # lr * |m_hat / sqrt(v_hat)| plus the rounding of the parameter
        assert np.all(np.abs(mv_new[P:] - st.v) <= 1e-5 * st.v + 1e-30), f"step {k}: second moment"
        upd = lr * np.abs(st.m / (1 - b1 ** k)) / (np.sqrt(st.v / (1 - b2 ** k)) + eps)
        tol = 1e-5 * upd + 2.0 ** -23 * np.abs(theta_new)
        bad = np.abs(theta_new - q.flat()) > tol
        assert not bad.any(), f"step {k}: {int(bad.sum())} parameters off the Adam update"
        theta, mv = theta_new, mv_new
    print(f"[train step] {desc} n={n}: {steps} steps, worst element error / bound {worst:.3f}",
          flush=True)


def test_train_64_heads_at_width_128(dev):
    """The largest map lt_map_create accepts (64 heads at width 128, 512
    output slots) trains: its backward on a ragged batch matches the oracle's
    quantised backward (every layer in relative norm, the output layer's 512
    slot rows element by element), and one fused step updates the
    parameters."""
    import torch
    import paper_2605_04017_amd as lt
    n = 65533   # the bound's batch size, with a ragged tail
    heads = 64
    rays = synth.config_rays(2, n)
    p = make_params(mlp.MapDesc(128, 3, heads, mlp.ACT_TANH), 564, rays)
    m = gpu_map(p, dev)
    r = to_dev(rays, dev)
    o, ws = lt.lt_map_forward_train(m, r)
    d_out = np.random.default_rng(64).normal(0, 1e-3, (6 * heads, n)).astype(np.float32)
    g = lt.lt_map_backward(m, torch.from_numpy(d_out).to(dev), ws)
    torch.cuda.synchronize()
    _, cache = mlp.forward_quantized_cache(p, mlp.features(rays, p))
    g_ref = mlp.backward_quantized(p, cache, d_out.T.astype(np.float64))
    worst = compare_grads(p, g.cpu().numpy(), g_ref)
    (gW, gb), (rW, rb) = split_layers(p, g.cpu().numpy())[-1], g_ref[-1]
    for a, ref, nm in ((gW, rW, "W"), (gb, rb, "b")):
        bound = GRAD_A * np.abs(ref) + GRAD_B * np.abs(ref).max()
        assert np.all(np.abs(a - ref) <= bound), (
            f"output layer {nm}: {int((np.abs(a - ref) > bound).sum())} elements outside the bound")
    t = {"valid": torch.ones((heads, n), dtype=torch.uint8, device=dev)}
    for k in ("x", "y", "dx", "dy", "throughput"):
        t[k] = torch.zeros((heads, n), dtype=torch.float32, device=dev)
    before = lt.lt_map_get_params(m).clone()
    lt.lt_map_train_step(m, r, t, {"lr": 1e-3, "step": 1}, lt.workspace(m, n))
    torch.cuda.synchronize()
    assert not torch.equal(before, lt.lt_map_get_params(m))
    print(f"[train] 64 heads x 128: worst relative layer error {worst:.2e}", flush=True)


def test_train_graph_replay_matches_eager(dev):
    """fit.TrainGraph (a run of lt_map_train_step calls recorded once in a
    HIP graph, learning rate and step read from device lt_train_sched
    entries) against eager lt_map_train_step calls on a twin map: after each
    of two replays of a three-step run on new batches, the parameters, Adam
    moments and per-step losses are bit-identical to the eager steps', with
    eager evaluations of the graph's map (which repack its weights) and host
    synchronisations between the replays.  Recorded before any eager step on
    its map."""
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd import fit as F
    n, heads, K = 3000, 3, 3
    rays_np = synth.config_rays(2, 2 * K * n)
    p = make_params(mlp.MapDesc(64, 3, heads, mlp.ACT_TANH), 777, rays_np)
    a, b = gpu_map(p, dev), gpu_map(p, dev)
    L = synth.config_lens(2)
    r_all, t_all = _trace_targets(L, rays_np, dev, heads)
    cfg = {"beta1": 0.9, "beta2": 0.999, "eps": 1e-8, "w_bce": 1.0, "w_l2": 2.0}
    g = F.TrainGraph(b, K, n, cfg, dev)
    ws = lt.workspace(a, n)
    loss_a = torch.zeros((K, 3), dtype=torch.float32, device=dev)
    for rep in range(2):
        lrs = [1e-3 * 0.7 ** (rep * K + k) for k in range(K)]
        for k in range(K):
            sl = slice((rep * K + k) * n, (rep * K + k + 1) * n)
            rb = {f: v[sl].contiguous() for f, v in r_all.items()}
            tb = {f: v[:, sl].contiguous() for f, v in t_all.items()}
            lt.lt_map_train_step(a, rb, tb, dict(cfg, lr=lrs[k], step=rep * K + k + 1), ws, loss_a[k])
            for f, v in g.rays.items():
                v[k * n:(k + 1) * n].copy_(rb[f])
            for f, v in g.targets.items():
                v[k].copy_(tb[f])
        loss_b = g.run(lrs, rep * K + 1)
        torch.cuda.synchronize()
        assert torch.equal(lt.lt_map_get_params(a), lt.lt_map_get_params(b)), f"run {rep}: parameters differ"
        assert torch.equal(lt.lt_map_adam_state(a), lt.lt_map_adam_state(b)), f"run {rep}: moments differ"
        assert torch.equal(loss_a, loss_b), f"run {rep}: losses differ"
        # eager work on the graph's map between replays
        oa = lt.lt_map_eval(a, lt.LT_BF16, rb)
        ob = lt.lt_map_eval(b, lt.LT_BF16, rb)
        torch.cuda.synchronize()
        for f in oa:
            assert torch.allclose(oa[f], ob[f], rtol=0.0, atol=0.0, equal_nan=True), f"run {rep}: eval {f} differs"
