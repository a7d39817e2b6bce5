"""Pins for the FP64 map reference (oracle/mlp.py): brute-force loops on tiny
networks, finite-difference gradients, closed forms of BCE and Adam, and the
rounding helpers against torch's own BF16 / FP8 conversions."""
import math

import numpy as np
import pytest

from oracle import mlp


def tiny(act=mlp.ACT_TANH, heads=2, width=3, depth=2, seed=0):
    d = mlp.MapDesc(width=width, depth=depth, n_heads=heads, activation=act)
    p = mlp.init_params(d, seed)
    rng = np.random.default_rng(seed + 1)
    for b in p.b:
        b[:] = rng.normal(0, 0.3, b.shape)
    p.in_shift = rng.normal(0, 0.1, 6)
    p.in_scale = rng.uniform(0.5, 2.0, 6)
    p.out_shift = rng.normal(0, 1, (heads, 5))
    p.out_scale = rng.uniform(0.5, 2, (heads, 5))
    return p


def loop_forward(p, x):
    """Scalar loops, one neuron at a time."""
    h = list(x)
    L = len(p.W)
    for li in range(L):
        W, b = p.W[li], p.b[li]
        z = []
        for o in range(W.shape[0]):
            s = b[o]
            for i in range(W.shape[1]):
                s += W[o, i] * h[i]
            z.append(s)
        if li < L - 1:
            h = [math.tanh(v) if p.desc.activation == mlp.ACT_TANH else max(v, 0.0) for v in z]
        else:
            h = z
    return np.array(h)


@pytest.mark.parametrize("act", [mlp.ACT_TANH, mlp.ACT_RELU])
def test_forward_matches_loops(act):
    p = tiny(act)
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1, (7, 6))
    o, _ = mlp.forward(p, x)
    for r in range(7):
        assert np.allclose(o[r], loop_forward(p, x[r]), atol=1e-13, rtol=0)


def test_features_and_decode():
    p = tiny(heads=2)
    rays = {"x": np.array([1.0, 2.0], np.float32), "y": np.array([0.5, -1], np.float32),
            "dx": np.array([0.1, 0.2], np.float32), "dy": np.array([0, 0.3], np.float32),
            "dz": np.array([-0.99, -0.9], np.float32), "lambda_nm": np.array([500, 600], np.float32)}
    f = mlp.features(rays, p)
    assert abs(f[1, 5] - (600 - p.in_shift[5]) * p.in_scale[5]) < 1e-12
    o = np.zeros((2, 12))
    o[0, 0], o[1, 0] = 1.0, -1.0      # head 0: ray 0 valid, ray 1 not
    o[:, 6] = 0.0                      # head 1: logit 0 -> not valid (strict >)
    o[0, 3] = (0.6 - p.out_shift[0, 2]) / p.out_scale[0, 2]
    o[0, 4] = (0.0 - p.out_shift[0, 3]) / p.out_scale[0, 3]
    d = mlp.decode(o, p)
    assert d["mask"].tolist() == [[1, 0], [0, 0]]
    assert abs(d["dx"][0, 0] - 0.6) < 1e-12 and abs(d["dz"][0, 0] + 0.8) < 1e-12
    assert np.isnan(d["x"][0, 1]) and d["throughput"][0, 1] == 0.0
    assert abs(d["x"][0, 0] - p.out_shift[0, 0]) < 1e-12  # o = 0 decodes to the shift


def test_bce_closed_form():
    p = tiny(heads=1)
    for b in p.b:
        b[:] = 0
    for W in p.W:
        W[:] = 0
    x = np.zeros((4, 6))
    valid = np.array([[1, 0, 1, 0]])
    (tot, bce, l2), _ = mlp.loss_and_grad(p, x, valid, np.zeros((1, 4, 5)))
    # logit 0 everywhere: BCE = log 2; outputs 0 = targets: no L2
    assert abs(bce - math.log(2)) < 1e-15 and l2 == 0.0 and tot == bce


@pytest.mark.parametrize("act", [mlp.ACT_TANH, mlp.ACT_RELU])
def test_gradient_finite_differences(act):
    p = tiny(act, heads=2, width=4, depth=3, seed=5)
    rng = np.random.default_rng(9)
    n = 6
    x = rng.normal(0, 1, (n, 6))
    valid = rng.integers(0, 2, (2, n))
    t = rng.normal(0, 1, (2, n, 5))
    _, grads = mlp.loss_and_grad(p, x, valid, t, 1.0, 0.7)
    g = mlp.grads_flat(grads)
    theta = p.flat()
    for k in rng.choice(theta.size, 40, replace=False):
        h = 1e-6 * max(1.0, abs(theta[k]))
        q = p.copy()
        th = theta.copy()
        th[k] += h
        q.set_flat(th)
        lp = mlp.loss_and_grad(q, x, valid, t, 1.0, 0.7)[0][0]
        th[k] -= 2 * h
        q.set_flat(th)
        lm = mlp.loss_and_grad(q, x, valid, t, 1.0, 0.7)[0][0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_adam_first_step_closed_form():
    p = tiny(heads=1)
    st = mlp.adam_init(p)
    theta0 = p.flat()
    g = np.random.default_rng(1).normal(0, 1e-3, theta0.size)
    mlp.adam_step(p, g, st, lr=1e-2, eps=1e-8)
    # bias-corrected first step: m_hat = g, v_hat = g^2
    expect = theta0 - 1e-2 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p.flat(), expect, atol=1e-15, rtol=1e-12)


def test_adam_matches_textbook_loop():
    p = tiny(heads=1)
    st = mlp.adam_init(p)
    th = p.flat().copy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    rng = np.random.default_rng(2)
    for k in range(1, 6):
        g = rng.normal(0, 1, th.size)
        mlp.adam_step(p, g, st, lr=1e-3, beta1=0.8, beta2=0.99, eps=1e-7)
        for i in range(th.size):
            m[i] = 0.8 * m[i] + 0.2 * g[i]
            v[i] = 0.99 * v[i] + 0.01 * g[i] * g[i]
            th[i] -= 1e-3 * (m[i] / (1 - 0.8 ** k)) / (math.sqrt(v[i] / (1 - 0.99 ** k)) + 1e-7)
    assert np.allclose(p.flat(), th, atol=1e-14, rtol=0)


def test_round_bf16_against_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 100000), rng.normal(0, 1e-30, 1000),
                        np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, 65504.0])])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.round_bf16(x), ref)
    assert mlp.round_bf16(np.array([1 + 2 ** -8]))[0] == 1.0        # tie to even
    assert mlp.round_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


def test_round_fp8_against_torch_and_code_table():
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("torch without float8_e4m3fn")
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8).view(torch.float8_e4m3fn)
    vals = codes.to(torch.float64).numpy()
    finite = vals[np.isfinite(vals)]
    assert np.abs(finite).max() == 448.0 and np.sum(np.isnan(vals)) == 2
    # every representable value rounds to itself
    assert np.array_equal(mlp.round_fp8_e4m3(finite), finite)
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(0, 30, 50000), rng.normal(0, 0.01, 50000),
                        rng.uniform(-448, 448, 20000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(mlp.round_fp8_e4m3(x), ref)
    assert mlp.round_fp8_e4m3(np.array([1000.0]))[0] == 448.0  # saturates


def test_quantized_forward_close_to_fp64():
    d = mlp.MapDesc(width=32, depth=4, n_heads=3)
    p = mlp.init_params(d, 11)
    x = np.random.default_rng(5).normal(0, 1, (500, 6))
    o, _ = mlp.forward(p, x)
    ob = mlp.forward_quantized(p, x, "bf16")
    o8 = mlp.forward_quantized(p, x, "fp8")
    eb = np.abs(ob - o).max()
    e8 = np.abs(o8 - o).max()
    assert eb < 0.05 and e8 < 0.3 and eb < e8


@pytest.mark.parametrize("act", [mlp.ACT_TANH, mlp.ACT_RELU])
def test_quantized_gradient_close_to_exact(act):
    """The BF16-rounding backward differs from exact backprop only by BF16
    rounding (a dropped term or a transposed operand would not).  ReLU
    differs more: rounding moves some pre-activations across 0, which
    switches units on or off."""
    d = mlp.MapDesc(32, 3, 2, act)
    p = mlp.init_params(d, 3)
    rng = np.random.default_rng(0)
    x = rng.normal(0, 1, (500, 6))
    v = rng.integers(0, 2, (2, 500))
    t = rng.normal(0, 1, (2, 500, 5))
    (l, _, _), g = mlp.loss_and_grad(p, x, v, t)
    (lq, _, _), gq = mlp.loss_and_grad_quantized(p, x, v, t)
    assert abs(l - lq) < 1e-3 * l
    tol = 2e-2 if act == mlp.ACT_TANH else 1e-1
    for (dW, db), (qW, qb) in zip(g, gq):
        assert np.linalg.norm(dW - qW) <= tol * np.linalg.norm(dW)
        assert np.linalg.norm(db - qb) <= tol * np.linalg.norm(db) + 1e-12


# ---------------------------------------------------------------- cosine loss

def _cos_setup(n=50, H=2, seed=0):
    desc = mlp.MapDesc(32, 2, H, mlp.ACT_TANH)
    p = mlp.init_params(desc, seed)
    rng = np.random.default_rng(seed)
    p.out_shift = rng.normal(0, 0.05, (H, 5))
    p.out_scale = rng.uniform(0.05, 0.3, (H, 5))
    o = rng.normal(0, 0.5, (n, 6 * H))
    t = rng.normal(0, 0.5, (H, n, 5))
    valid = rng.integers(0, 2, (H, n))
    return p, o, t, valid


def test_cosine_loss_zero_for_identical_directions():
    p, o, t, valid = _cos_setup()
    H, n = valid.shape
    oo = o.reshape(n, H, 6)
    t[..., 2] = oo[..., 3].T          # target direction = predicted direction
    t[..., 3] = oo[..., 4].T
    (tot, bce, reg), g = mlp.loss_terms(p, o, valid, t, 0.0, 0.0, 1.0)
    assert abs(reg) < 1e-13 and abs(tot - reg) < 1e-13
    gg = g.reshape(n, H, 6)
    assert np.abs(gg[..., 3:5]).max() < 1e-12


def test_cosine_loss_known_angle():
    """Target and prediction in the x-z plane, the prediction turned by
    theta: the loss is 1 - cos(theta) per valid ray."""
    H, n = 1, 5
    p = mlp.init_params(mlp.MapDesc(32, 2, H, mlp.ACT_TANH), 0)
    a = np.linspace(0.05, 0.4, n)
    theta = 0.1
    o = np.zeros((n, 6))
    o[:, 3] = np.sin(a + theta)       # out_shift 0, out_scale 1: raw = lens units
    t = np.zeros((H, n, 5))
    t[0, :, 2] = np.sin(a)
    valid = np.ones((H, n), int)
    (_, _, reg), _ = mlp.loss_terms(p, o, valid, t, 0.0, 0.0, 2.0)
    assert abs(reg - 2.0 * (1 - np.cos(theta))) < 1e-12


def test_cosine_loss_gradient_finite_differences():
    p, o, t, valid = _cos_setup(n=40)
    w = (0.7, 1.3, 2.1)
    _, g = mlp.loss_terms(p, o, valid, t, *w)
    rng = np.random.default_rng(3)
    for idx in rng.choice(o.size, 60, replace=False):
        i, j = divmod(int(idx), o.shape[1])
        h = 1e-6
        op, om = o.copy(), o.copy()
        op[i, j] += h
        om[i, j] -= h
        fd = (mlp.loss_terms(p, op, valid, t, *w)[0][0] - mlp.loss_terms(p, om, valid, t, *w)[0][0]) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6 * max(1.0, abs(fd)), (i, j, fd, g[i, j])


def test_cosine_loss_parameter_gradient():
    """loss_and_grad with the cosine term against central differences of
    the FP64 loss in the parameters."""
    rng = np.random.default_rng(4)
    desc = mlp.MapDesc(32, 3, 1, mlp.ACT_TANH)
    p = mlp.init_params(desc, 4)
    p.out_scale = np.array([[1.0, 1.0, 0.2, 0.2, 1.0]])
    x = rng.normal(0, 1, (30, 6))
    t = rng.normal(0, 0.5, (1, 30, 5))
    valid = rng.integers(0, 2, (1, 30))
    _, grads = mlp.loss_and_grad(p, x, valid, t, 1.0, 0.5, 1.5)
    flat = mlp.grads_flat(grads)
    theta = p.flat()
    for k in rng.choice(theta.size, 25, replace=False):
        h = 1e-6
        q = p.copy()
        th = theta.copy()
        th[k] += h
        q.set_flat(th)
        lp = mlp.loss_and_grad(q, x, valid, t, 1.0, 0.5, 1.5)[0][0]
        th[k] -= 2 * h
        q.set_flat(th)
        lm = mlp.loss_and_grad(q, x, valid, t, 1.0, 0.5, 1.5)[0][0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - flat[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, flat[k])


def test_forward_map_decode_flips_only_dz():
    """A forward map decodes the same exit rays as a sensor-side map with the
    same parameters except for the sign of dz (unit directions toward the
    sensor)."""
    import dataclasses
    import synth
    rays = synth.config_rays(1, 500)
    d0 = mlp.MapDesc(32, 2, 3, mlp.ACT_TANH)
    p0 = mlp.init_params(d0, 5)
    p1 = dataclasses.replace(p0, desc=dataclasses.replace(d0, forward=True))
    o = mlp.forward(p0, mlp.features(rays, p0))[0]
    a, b = mlp.decode(o, p0, rays), mlp.decode(o, p1, rays)
    for k in ("logit", "mask", "x", "y", "dx", "dy", "throughput"):
        assert np.array_equal(a[k], b[k], equal_nan=True)
    ok = a["mask"] == 1
    assert np.array_equal(-a["dz"][ok], b["dz"][ok])
    assert np.all(b["dz"][ok] >= 0)
    s2 = b["dx"][ok] ** 2 + b["dy"][ok] ** 2
    assert np.allclose(b["dz"][ok] ** 2, np.maximum(0.0, 1.0 - s2), rtol=0, atol=1e-12)
