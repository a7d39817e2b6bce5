"""Pins for the oracle's reduced-precision network (oracle/mlp.py:
forward_quantized in its BF16 evaluation (folded for tanh), BF16 training
and FP8 forms, forward_quantized_cache, backward_quantized), which every
BF16 / FP8 parity test of the GPU kernels is measured against.

Three kinds of pin, none of which reuses the oracle's rounding code:
  * independent scalar-loop networks, one neuron at a time, that round with
    torch's BF16 conversion and with an FP8 E4M3 rounding done by nearest-
    even search in torch's FP8 code table, at the rounding points of the
    kernels (split hi + lo BF16 input and output layers, BF16 or FP8 hidden
    layers, one rounding per activation); the oracle must agree to FP64
    summation order;
  * special cases with a plain definition: with BF16-exact (and FP8-exact)
    parameters and inputs the split terms vanish and the network is the FP64
    network with every activation rounded exactly once; for the folded BF16
    evaluation of a tanh map, with weights whose folded copies are BF16-exact,
    it is the FP64 tanh network in which every hidden value passes through
    r = (1 - tanh z) / 2 rounded exactly once;
  * the accuracy the split layers promise: hi + lo BF16 inputs and weights
    reproduce the exact layer to 3.1 * 2^-16 of the sum of |x_i W_ji|, split
    weights on BF16 activations to 2.1 * 2^-16 of it (the dropped terms
    x_lo W_lo and the rounding of each lo part are each below 2^-16 of a
    product).
A mutation test then replaces one rounding or split step of the oracle at a
time (a dropped split term, an extra or a missing rounding, an unrounded
weight, a wrong derivative) and checks that some pin fails for each.
"""
import math

import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")


# ------------------------------------------------ independent rounding ----

def bf(v):
    """Round to BF16 through torch (the value is first an FP32 number, as in
    the kernels' registers); float64 out."""
    a = torch.from_numpy(np.asarray(v, np.float64).astype(np.float32))
    return a.to(torch.bfloat16).to(torch.float64).numpy()


def _fp8_table():
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    vals = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    fin = np.isfinite(vals)
    v, c = vals[fin], np.arange(256)[fin]
    order = np.argsort(v, kind="stable")
    v, c = v[order], c[order]
    keep = np.r_[True, v[1:] != v[:-1]]   # +0 and -0 collapse to one entry
    return v[keep], c[keep]


if hasattr(torch, "float8_e4m3fn"):
    F8_VALS, F8_CODES = _fp8_table()


def f8(v):
    """OCP E4M3 round to nearest, ties to the even code, saturating at
    +-448: nearest neighbour search in the table of representable values."""
    v = np.clip(np.asarray(v, np.float64), -448.0, 448.0)
    i = np.clip(np.searchsorted(F8_VALS, v), 1, F8_VALS.size - 1)
    lo, hi = F8_VALS[i - 1], F8_VALS[i]
    dlo, dhi = v - lo, hi - v
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (F8_CODES[i] % 2 == 0))
    return np.where(pick_hi, hi, lo)


def pow2_below(amax, target):
    return 2.0 ** math.floor(math.log2(target / amax))


def act(z, kind):
    return math.tanh(z) if kind == mlp.ACT_TANH else max(z, 0.0)


# --------------------------------------------- scalar-loop references ----

K2 = float(np.float32(2.0 / math.log(2.0)))   # 2 log2 e as an FP32 number


def f32mul(a, b):
    """a * b with FP32 operands and one FP32 rounding."""
    return float(np.float32(np.float32(a) * np.float32(b)))


def loop_forward_folded(p, x):
    """One ray through the BF16 evaluation of a tanh map, neuron by neuron:
    every hidden value is r = (1 - tanh z) / 2, rounded once; the layers
    carry k = 2 log2 e and the map h = 1 - 2 r (u = k z, r = 1 / (1 + 2^u)),
    with each folded weight, k W0 (split hi + lo) and BF16(-2 k W), and each
    k b formed in FP32 as the packer forms them."""
    L = len(p.W)
    x_hi = bf(x)
    x_lo = bf(x - x_hi)
    kW0 = np.vectorize(lambda w: f32mul(w, K2))(p.W[0])
    W0_hi = bf(kW0)
    W0_lo = bf(kW0 - W0_hi)
    u = []
    for j in range(p.W[0].shape[0]):
        s = f32mul(p.b[0][j], K2)
        for i in range(6):
            s += x_hi[i] * W0_hi[j, i] + x_lo[i] * W0_hi[j, i] + x_hi[i] * W0_lo[j, i]
        u.append(s)
    r = bf(np.array([(1.0 - math.tanh(v / K2)) / 2.0 for v in u]))
    for li in range(1, L - 1):
        W = p.W[li]
        un = []
        for j in range(W.shape[0]):
            # k (sum_i W'_ji (1 - 2 r_i) + b_j) with W'_ji = BF16(-2 k W_ji) / (-2 k)
            s = f32mul(p.b[li][j], K2)
            for i in range(W.shape[1]):
                wq = bf(f32mul(W[j, i], -2.0 * K2))
                s += wq * r[i] - 0.5 * wq
            un.append(s)
        r = bf(np.array([(1.0 - math.tanh(v / K2)) / 2.0 for v in un]))
    Wo = p.W[L - 1]
    Wo_hi = bf(Wo)
    Wo_lo = bf(Wo - Wo_hi)
    o = []
    for k in range(Wo.shape[0]):
        s = p.b[L - 1][k]
        for j in range(Wo.shape[1]):
            s += (1.0 - 2.0 * r[j]) * (Wo_hi[k, j] + Wo_lo[k, j])
        o.append(s)
    return np.array(o)


def loop_forward(p, x, mode):
    """One ray through the quantised network, neuron by neuron.  mode "bf16"
    is the BF16 evaluation (folded for tanh maps), "bf16_train" the training
    forward, "fp8" the FP8 evaluation."""
    kind = p.desc.activation
    if mode == "bf16" and kind == mlp.ACT_TANH:
        return loop_forward_folded(p, x)
    L = len(p.W)
    x_hi = bf(x)
    x_lo = bf(x - x_hi)
    W0_hi = bf(p.W[0])
    W0_lo = bf(p.W[0] - W0_hi)
    z = []
    for j in range(p.W[0].shape[0]):
        s = p.b[0][j]
        for i in range(6):
            s += x_hi[i] * W0_hi[j, i] + x_lo[i] * W0_hi[j, i] + x_hi[i] * W0_lo[j, i]
        z.append(s)
    if mode == "fp8":
        for li in range(1, L - 1):
            W = p.W[li]
            sw = pow2_below(np.abs(W).max(), 448.0)
            sh = 256.0 if kind == mlp.ACT_TANH else 1.0
            hq = f8(np.array([act(v, kind) * sh for v in z]))
            Wq = f8(W * sw)
            zn = []
            for j in range(W.shape[0]):
                s = 0.0
                for i in range(W.shape[1]):
                    s += hq[i] * Wq[j, i]
                zn.append(s / (sw * sh) + p.b[li][j])
            z = zn
        h = bf(np.array([act(v, kind) for v in z]))
    else:
        h = bf(np.array([act(v, kind) for v in z]))
        for li in range(1, L - 1):
            Wb = bf(p.W[li])
            zn = []
            for j in range(Wb.shape[0]):
                s = p.b[li][j]
                for i in range(Wb.shape[1]):
                    s += h[i] * Wb[j, i]
                zn.append(s)
            h = bf(np.array([act(v, kind) for v in zn]))
    Wo = p.W[L - 1]
    Wo_hi = bf(Wo)
    Wo_lo = bf(Wo - Wo_hi)
    o = []
    for k in range(Wo.shape[0]):
        s = p.b[L - 1][k]
        for j in range(Wo.shape[1]):
            s += h[j] * Wo_hi[k, j] + h[j] * Wo_lo[k, j]
        o.append(s)
    return np.array(o)


def loop_backward(p, X, D):
    """Chain rule over a batch X (n, 6) for output gradients D (n, 6H), ray
    by ray and neuron by neuron, with the training kernels' rounding points:
    the output gradient split hi + lo, every hidden pre-activation gradient
    rounded once to BF16 after the derivative (taken from the stored BF16
    activation), BF16 weights in the transpose products, split inputs for
    the first layer's weight gradient."""
    kind = p.desc.activation
    L = len(p.W)
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in zip(p.W, p.b)]
    for r in range(X.shape[0]):
        # forward of the training kernels, keeping the stored activations
        x = X[r]
        x_hi = bf(x)
        x_lo = bf(x - x_hi)
        W0_hi = bf(p.W[0])
        W0_lo = bf(p.W[0] - W0_hi)
        z = [p.b[0][j] + sum(x_hi[i] * W0_hi[j, i] + x_lo[i] * W0_hi[j, i] + x_hi[i] * W0_lo[j, i]
                             for i in range(6)) for j in range(p.W[0].shape[0])]
        hs = [bf(np.array([act(v, kind) for v in z]))]
        for li in range(1, L - 1):
            Wb = bf(p.W[li])
            z = [p.b[li][j] + sum(hs[-1][i] * Wb[j, i] for i in range(Wb.shape[1]))
                 for j in range(Wb.shape[0])]
            hs.append(bf(np.array([act(v, kind) for v in z])))
        d_hi = bf(D[r])
        d = d_hi + bf(D[r] - d_hi)
        gW, gb = grads[L - 1]
        for k in range(d.size):
            gb[k] += d[k]
            for j in range(hs[-1].size):
                gW[k, j] += d[k] * hs[-1][j]
        Wb = bf(p.W[L - 1])
        delta = [sum(d[k] * Wb[k, j] for k in range(d.size)) for j in range(Wb.shape[1])]
        for li in range(L - 2, -1, -1):
            h = hs[li]
            der = [(1.0 - v * v) if kind == mlp.ACT_TANH else (1.0 if v > 0 else 0.0) for v in h]
            db = bf(np.array([delta[j] * der[j] for j in range(h.size)]))
            prev = (x_hi + x_lo) if li == 0 else hs[li - 1]
            gW, gb = grads[li]
            for j in range(h.size):
                gb[j] += db[j]
                for i in range(prev.size):
                    gW[j, i] += db[j] * prev[i]
            if li > 0:
                Wt = bf(p.W[li])
                delta = [sum(db[j] * Wt[j, i] for j in range(h.size)) for i in range(Wt.shape[1])]
    return grads


# ------------------------------------------------------------- inputs ----

def net(width=16, depth=3, heads=2, act_kind=mlp.ACT_TANH, seed=0, bias=0.3):
    d = mlp.MapDesc(width=width, depth=depth, n_heads=heads, activation=act_kind)
    p = mlp.init_params(d, seed)
    rng = np.random.default_rng(seed + 100)
    for li, W in enumerate(p.W):
        # spread the weights over several binades so FP8 scales and
        # subnormals are exercised
        W *= np.exp2(rng.integers(-3, 3, W.shape))
        p.b[li] = rng.normal(0, bias, p.b[li].shape)
    return p


def inputs(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 1.2, (n, 6))


# --------------------------------------------------------------- pins ----

def pin_forward_loops(modes=("bf16", "bf16_train", "fp8")):
    for mode in modes:
        for kind in (mlp.ACT_TANH, mlp.ACT_RELU):
            p = net(act_kind=kind, seed=3 + kind)
            X = inputs(24, 7)
            o = mlp.forward_quantized(p, X, mode)
            for r in range(X.shape[0]):
                ref = loop_forward(p, X[r], mode)
                assert np.allclose(o[r], ref, rtol=0, atol=1e-12), (mode, kind, r,
                                                                     np.abs(o[r] - ref).max())


def pin_exact_parameters_round_once():
    """BF16-exact parameters and inputs: the oracle's BF16 network is the
    FP64 network with each activation rounded once (no split term survives);
    FP8-exact scaled hidden weights: the FP8 network is the FP64 network with
    each hidden activation rounded once to E4M3 at scale 2^8."""
    for kind in (mlp.ACT_TANH, mlp.ACT_RELU):
        p = net(act_kind=kind, seed=11)
        for li in range(len(p.W)):
            p.W[li] = bf(p.W[li])
            p.b[li] = bf(p.b[li])
        X = bf(inputs(20, 12))
        o = mlp.forward_quantized(p, X, "bf16_train")
        for r in range(X.shape[0]):
            h = X[r]
            for li in range(len(p.W)):
                z = p.W[li] @ h + p.b[li]
                h = bf(np.array([act(v, kind) for v in z])) if li < len(p.W) - 1 else z
            assert np.allclose(o[r], h, rtol=0, atol=1e-12), ("bf16", kind, r)
        # FP8: hidden weights w * 2^-sw_exp with w on the E4M3 grid
        q = p.copy()
        for li in range(1, len(q.W) - 1):
            sw = pow2_below(np.abs(q.W[li]).max(), 448.0)
            q.W[li] = f8(q.W[li] * sw) / sw
        o8 = mlp.forward_quantized(q, X, "fp8")
        sh = 256.0 if kind == mlp.ACT_TANH else 1.0
        for r in range(X.shape[0]):
            z = q.W[0] @ X[r] + q.b[0]
            for li in range(1, len(q.W) - 1):
                hq = f8(np.array([act(v, kind) for v in z]) * sh) / sh
                z = q.W[li] @ hq + q.b[li]
            h = bf(np.array([act(v, kind) for v in z]))
            ref = q.W[-1] @ h + q.b[-1]   # BF16-exact output weights: no lo part
            assert np.allclose(o8[r], ref, rtol=0, atol=1e-12), ("fp8", kind, r)


def pin_folded_round_once():
    """BF16 evaluation of a tanh map with weights and inputs chosen so that
    every folded copy is exact (k W0, k b and BF16(-2 k W) equal their FP64
    products, split parts vanish): the network is the FP64 tanh network in
    which every hidden value h = tanh z is replaced by 1 - 2 BF16((1 - h) / 2),
    the output layer taking h in that form."""
    p = net(seed=61)
    # weights w = q / (-2 k) for q on a coarse binary grid, so that
    # FP32(w * (-2 k)) == q exactly (the grid is checked, not assumed)
    rng = np.random.default_rng(62)
    for li in range(len(p.W)):
        q = rng.integers(-8, 9, p.W[li].shape) / 8.0
        W = np.float32(q) / np.float32(-2.0 * K2)
        W = W.astype(np.float64)
        back = np.vectorize(lambda w: f32mul(w, -2.0 * K2))(W)
        keep = (back == q) & (np.vectorize(lambda w: f32mul(w, K2))(W) == -q / 2)
        p.W[li] = np.where(keep, W, 0.0)
        qb = rng.integers(-8, 9, p.b[li].shape) / 8.0
        b = (np.float32(qb) / np.float32(K2)).astype(np.float64)
        okb = np.vectorize(lambda v: f32mul(v, K2))(b) == qb
        p.b[li] = np.where(okb, b, 0.0)
    # the output layer splits its weights: make them BF16-exact
    p.W[-1] = bf(p.W[-1])
    p.W[-1] = np.where(bf(p.W[-1] - bf(p.W[-1])) == 0, p.W[-1], 0.0)
    X = bf(inputs(20, 63))
    o = mlp.forward_quantized(p, X, "bf16")
    for r_i in range(X.shape[0]):
        h = X[r_i]
        for li in range(len(p.W)):
            z = p.W[li] @ h + p.b[li]
            if li < len(p.W) - 1:
                rq = bf(np.array([(1.0 - math.tanh(v)) / 2.0 for v in z]))
                h = 1.0 - 2.0 * rq
            else:
                h = z
        assert np.allclose(o[r_i], h, rtol=0, atol=1e-12), ("folded", r_i, np.abs(o[r_i] - h).max())


def pin_scale_is_an_fp32_product():
    """The folded weights are FP32 products (the packer multiplies FP32 values
    in FP32): the oracle's products equal torch's FP32 multiplication, which
    differs from the FP64 product on most of these values."""
    rng = np.random.default_rng(81)
    a = rng.normal(0, 3, 5000)
    for sc in (mlp.K_TANH, -2.0 * mlp.K_TANH):
        ref = (torch.from_numpy(a.astype(np.float32)) * torch.tensor(sc, dtype=torch.float32)).double().numpy()
        assert np.array_equal(mlp.scale_f32(a, sc), ref)
        assert np.mean(ref != a.astype(np.float32).astype(np.float64) * sc) > 0.5


def pin_folded_close_to_unfolded():
    """The folded and unfolded BF16 evaluations of one tanh network differ
    only by where BF16 rounds (r instead of tanh z, BF16(-2 k W) instead of
    BF16(W)): both stay within BF16 accuracy of the FP64 network and of each
    other, while a dropped bias correction or a missing factor would not."""
    p = net(seed=71, width=32, depth=4, heads=2)
    X = inputs(400, 72)
    o64, _ = mlp.forward(p, X)
    of = mlp.forward_quantized(p, X, "bf16")
    ou = mlp.forward_quantized(p, X, "bf16_train")
    scale = np.abs(o64).max()
    assert np.abs(of - o64).max() < 0.05 * scale and np.abs(ou - o64).max() < 0.05 * scale
    assert np.abs(of - ou).max() < 0.05 * scale


def pin_split_layer_accuracy():
    rng = np.random.default_rng(21)
    X = rng.normal(0, 1, (400, 6)) * np.exp2(rng.integers(-4, 4, (400, 6)))
    W0 = rng.normal(0, 1, (32, 6)) * np.exp2(rng.integers(-4, 4, (32, 6)))
    b0 = rng.normal(0, 1, 32)
    z, (x_hi, x_lo) = mlp.input_layer_split(X, W0, b0)
    exact = X @ W0.T + b0
    absum = np.abs(X) @ np.abs(W0).T
    assert np.all(np.abs(z - exact) <= 3.1 * 2.0 ** -16 * absum), "input layer split"
    assert np.array_equal(x_hi, bf(X)) and np.array_equal(x_lo, bf(X - bf(X)))
    H = bf(np.tanh(rng.normal(0, 1, (400, 32))))
    Wo = rng.normal(0, 1, (12, 32)) * np.exp2(rng.integers(-4, 4, (12, 32)))
    bo = rng.normal(0, 1, 12)
    o = mlp.output_layer_split(H, Wo, bo)
    assert np.all(np.abs(o - (H @ Wo.T + bo)) <= 2.1 * 2.0 ** -16 * (np.abs(H) @ np.abs(Wo).T)), \
        "output layer split"


def pin_training_forward():
    p = net(seed=31)
    X = inputs(50, 32)
    o, (x_hi, x_lo, hs) = mlp.forward_quantized_cache(p, X)
    assert np.array_equal(o, mlp.forward_quantized(p, X, "bf16_train"))
    assert len(hs) == p.desc.depth and all(np.array_equal(h, bf(h)) for h in hs)


def pin_backward_loops():
    for kind in (mlp.ACT_TANH, mlp.ACT_RELU):
        p = net(width=12, depth=3, heads=2, act_kind=kind, seed=41 + kind)
        X = inputs(10, 42)
        D = np.random.default_rng(43).normal(0, 1, (10, 12))
        _, cache = mlp.forward_quantized_cache(p, X)
        got = mlp.backward_quantized(p, cache, D)
        ref = loop_backward(p, X, D)
        for li, ((gW, gb), (rW, rb)) in enumerate(zip(got, ref)):
            assert np.allclose(gW, rW, rtol=0, atol=1e-12 * max(1.0, np.abs(rW).max())), (kind, li, "W")
            assert np.allclose(gb, rb, rtol=0, atol=1e-12 * max(1.0, np.abs(rb).max())), (kind, li, "b")


ALL_PINS = (pin_forward_loops, pin_exact_parameters_round_once, pin_folded_round_once,
            pin_scale_is_an_fp32_product, pin_folded_close_to_unfolded, pin_split_layer_accuracy,
            pin_training_forward, pin_backward_loops)


@pytest.mark.skipif(not hasattr(torch, "float8_e4m3fn"), reason="torch without float8_e4m3fn")
@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


def test_fp8_table_rounding_against_the_oracle_definition():
    """The test's table-search E4M3 rounding and the oracle's log2-based one
    agree (two independent readings of the OCP format)."""
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.normal(0, 50, 20000), rng.normal(0, 1e-2, 20000), F8_VALS,
                        (F8_VALS[1:] + F8_VALS[:-1]) / 2, [500.0, -1000.0]])
    assert np.array_equal(f8(v), mlp.round_fp8_e4m3(v))


# ------------------------------------------------------------ mutants ----
# Each replaces one step of the oracle with a plausible mistake.

def _input_drop_xlo(xhat, W0, b0):
    x_hi, x_lo = mlp.split_bf16(xhat)
    W_hi, W_lo = mlp.split_bf16(W0)
    return x_hi @ W_hi.T + x_hi @ W_lo.T + b0, (x_hi, x_lo)


def _input_drop_wlo(xhat, W0, b0):
    x_hi, x_lo = mlp.split_bf16(xhat)
    W_hi, _ = mlp.split_bf16(W0)
    return x_hi @ W_hi.T + x_lo @ W_hi.T + b0, (x_hi, x_lo)


def _input_no_split(xhat, W0, b0):
    x_hi, x_lo = mlp.split_bf16(xhat)
    return x_hi @ mlp.round_bf16(W0).T + b0, (x_hi, x_lo)


def _output_drop_wlo(h, Wo, bo):
    return h @ mlp.round_bf16(Wo).T + bo


def _activation_round_z_too(z, kind):
    return mlp.round_bf16(mlp.act(mlp.round_bf16(z), kind))


def _activation_unrounded(z, kind):
    return mlp.act(z, kind)


def _hidden_unrounded_weights(h, W, b):
    return h @ W.T + b


def _fp8_double_rounding(z_prev, W, b, sw, sh, kind):
    hq = mlp.round_fp8_e4m3(mlp.round_bf16(mlp.act(z_prev, kind)) * sh)
    return (hq @ mlp.round_fp8_e4m3(W * sw).T) / (sw * sh) + b


def _fp8_unscaled_weights(z_prev, W, b, sw, sh, kind):
    hq = mlp.round_fp8_e4m3(mlp.act(z_prev, kind) * sh)
    return (hq @ mlp.round_fp8_e4m3(W).T) / sh + b


def _grad_no_split(d_out):
    return mlp.round_bf16(d_out)


def _grad_unrounded(delta, h, kind):
    dphi = 1.0 - h * h if kind == mlp.ACT_TANH else (h > 0).astype(np.float64)
    return delta * dphi


def _grad_wrong_derivative(delta, h, kind):
    dphi = 1.0 - h if kind == mlp.ACT_TANH else (h > 0).astype(np.float64)
    return mlp.round_bf16(delta * dphi)


def _transpose_unrounded(W):
    return W


def _folded_act_unrounded(u):
    return 1.0 / (1.0 + np.exp2(u))


def _folded_act_natural_exp(u):
    return mlp.round_bf16(1.0 / (1.0 + np.exp(u)))


def _folded_hidden_no_bias_correction(r, W, b):
    Wq = mlp.round_bf16(mlp.scale_f32(W, -2.0 * mlp.K_TANH))
    return r @ Wq.T + mlp.scale_f32(b, mlp.K_TANH)


def _folded_hidden_unrounded_weights(r, W, b):
    Wq = mlp.scale_f32(W, -2.0 * mlp.K_TANH)
    return r @ Wq.T + mlp.scale_f32(b, mlp.K_TANH) - 0.5 * Wq.sum(1)


def _folded_output_no_bias_correction(r, Wo, bo):
    W_hi, W_lo = mlp.split_bf16(Wo)
    return r @ (-2.0 * W_hi).T + r @ (-2.0 * W_lo).T + bo


def _scale_f64(a, s):
    return np.asarray(a, np.float64) * s


MUTANTS = [("input_layer_split", _input_drop_xlo), ("input_layer_split", _input_drop_wlo),
           ("input_layer_split", _input_no_split), ("output_layer_split", _output_drop_wlo),
           ("activation_bf16", _activation_round_z_too), ("activation_bf16", _activation_unrounded),
           ("hidden_layer_bf16", _hidden_unrounded_weights), ("hidden_layer_fp8", _fp8_double_rounding),
           ("hidden_layer_fp8", _fp8_unscaled_weights), ("output_grad_split", _grad_no_split),
           ("hidden_grad_bf16", _grad_unrounded), ("hidden_grad_bf16", _grad_wrong_derivative),
           ("transpose_weights_bf16", _transpose_unrounded),
           ("activation_folded_bf16", _folded_act_unrounded),
           ("activation_folded_bf16", _folded_act_natural_exp),
           ("hidden_layer_folded_bf16", _folded_hidden_no_bias_correction),
           ("hidden_layer_folded_bf16", _folded_hidden_unrounded_weights),
           ("output_layer_folded", _folded_output_no_bias_correction), ("scale_f32", _scale_f64)]


@pytest.mark.skipif(not hasattr(torch, "float8_e4m3fn"), reason="torch without float8_e4m3fn")
@pytest.mark.parametrize("name,mutant", MUTANTS, ids=[m[1].__name__.lstrip("_") for m in MUTANTS])
def test_each_mutation_fails_a_pin(monkeypatch, name, mutant):
    monkeypatch.setattr(mlp, name, mutant)
    failed = []
    for pin in ALL_PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin catches the mutation {mutant.__name__} of {name}"
