"""FP64 reference of the precomputed lens transport map (TEST INFRASTRUCTURE).

The map follows Sec. 4.2 of the paper ("Neural Ray Masking"): per light path
a classifier g(x) decides whether the input ray is valid and a regressor
f(x) gives the exit ray and its Fresnel throughput; the model outputs f(x)
where g(x) = 1 and nothing otherwise.  Hidden layers use tanh for C^1
smoothness (Sec. 4.2, "C^1 Continuous Network"); a ReLU variant is kept for
the small doublet workload.  Here the classifier logit and the regression
outputs of every path are heads of one shared trunk:

    xhat = (input - in_shift) * in_scale                     (6 features)
    h_0 = xhat;  h_l = phi(W_l h_{l-1} + b_l),  l = 1..depth
    o = W_out h_depth + b_out                                (6 per head)
    head p: logit = o[6p], mask = logit > 0,
            (x, y, dx, dy, I) = out_shift + out_scale * o[6p+1 .. 6p+5],
            dz = -sqrt(1 - dx^2 - dy^2);  mask = 0 gives NaN fields, I = 0.

Training loss (per head, averaged over heads): binary cross-entropy of the
logit against the traced validity plus the squared error of the normalised
regression outputs on valid rays only (the regressor only has to fit the
valid region, Sec. 4.2):

    L = mean_p [ w_bce/N sum_i BCE(logit_ip, v_ip)
               + w_l2/(5N) sum_i v_ip sum_d (o_ipd - t_ipd)^2 ]

Adam follows Kingma and Ba (2015) with bias correction.

The quantised forward (`forward_quantized`) rounds exactly where the GPU
kernels round -- BF16 round-to-nearest-even for weights and activations,
split hi/lo BF16 for the input layer and the output layer, OCP FP8 E4M3
(bias 7, max 448, round-to-nearest-even, subnormals, saturating) with
power-of-two per-layer scales for the hidden layers in FP8 mode -- and
otherwise computes in FP64, so it pins the kernels up to FP32 accumulation
order.  BF16 evaluation of a tanh map runs the folded form of the same
network (`forward_folded_bf16`): with k = 2 log2 e, r = 1 / (1 + 2^(k z))
and tanh z = 1 - 2 r, the scale k and the affine map move into the weights,
and the rounded activation is r instead of tanh z.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List

import numpy as np

ACT_TANH = 0
ACT_RELU = 1
N_OUT = 6  # logit, x, y, dx, dy, throughput


@dataclasses.dataclass
class MapDesc:
    width: int = 128
    depth: int = 5          # hidden layers
    n_heads: int = 1
    activation: int = ACT_TANH
    canonical: bool = False  # symmetry-reduced input (Sec. 4.1), see canonical_frame
    forward: bool = False    # forward light tracing map (Sec. 3): exits travel toward the sensor, dz > 0


@dataclasses.dataclass
class MapParams:
    desc: MapDesc
    W: List[np.ndarray]       # W[0]: (width, 6), W[1..depth-1]: (width, width), W[depth]: (6H, width)
    b: List[np.ndarray]
    in_shift: np.ndarray      # (6,)
    in_scale: np.ndarray      # (6,)
    out_shift: np.ndarray     # (H, 5)
    out_scale: np.ndarray     # (H, 5)

    def flat(self) -> np.ndarray:
        """Parameter vector in the library's order: W0, b0, W1, b1, ..., Wout, bout
        (row-major, output index first)."""
        parts = []
        for W, b in zip(self.W, self.b):
            parts.append(W.reshape(-1))
            parts.append(b.reshape(-1))
        return np.concatenate(parts)

    def set_flat(self, v: np.ndarray):
        k = 0
        for li in range(len(self.W)):
            n = self.W[li].size
            self.W[li] = v[k:k + n].reshape(self.W[li].shape).astype(np.float64)
            k += n
            n = self.b[li].size
            self.b[li] = v[k:k + n].astype(np.float64)
            k += n
        assert k == v.size

    def copy(self) -> "MapParams":
        return MapParams(self.desc, [w.copy() for w in self.W], [b.copy() for b in self.b],
                         self.in_shift.copy(), self.in_scale.copy(), self.out_shift.copy(),
                         self.out_scale.copy())


def layer_shapes(desc: MapDesc):
    shapes = [(desc.width, 6)]
    shapes += [(desc.width, desc.width)] * (desc.depth - 1)
    shapes.append((N_OUT * desc.n_heads, desc.width))
    return shapes


def n_params(desc: MapDesc) -> int:
    return sum(o * i + o for (o, i) in layer_shapes(desc))


def init_params(desc: MapDesc, seed: int) -> MapParams:
    """Uniform Glorot initialisation, zero biases, identity normalisation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W, b = [], []
    for (o, i) in layer_shapes(desc):
        lim = math.sqrt(6.0 / (o + i))
        W.append(rng.uniform(-lim, lim, (o, i)))
        b.append(np.zeros(o))
    H = desc.n_heads
    return MapParams(desc, W, b, np.zeros(6), np.ones(6), np.zeros((H, 5)), np.ones((H, 5)))


def canonical_frame(rays: Dict[str, np.ndarray]):
    """Symmetry reduction of the input (Sec. 4.1, geometric simplification):
    rotate about the optical axis so the sensor point lies on the +x half
    line, then mirror in the plane through the axis and that point so the
    direction's y component is >= 0.  The map commutes with both, so the
    network only sees r >= 0, y = 0, dy >= 0 and the outputs are mapped back.

    Evaluated in float32 with one rounding per operation (the products,
    sums, square root and quotients below, in this order), as the kernels do,
    so both sides feed the network identical canonical inputs.  A sensor
    point on the axis keeps the identity rotation.  Returns (canonical rays
    (float32), c, s, flip) with c, s float32 and flip bool."""
    f32 = np.float32
    x, y = rays["x"].astype(f32), rays["y"].astype(f32)
    dx, dy = rays["dx"].astype(f32), rays["dy"].astype(f32)
    r = np.sqrt(x * x + y * y)
    pos = r > 0
    safe = np.where(pos, r, f32(1))
    c = np.where(pos, x / safe, f32(1)).astype(f32)
    s = np.where(pos, y / safe, f32(0)).astype(f32)
    dxr = c * dx + s * dy
    dyr = c * dy - s * dx
    flip = dyr < 0
    dyr = np.where(flip, -dyr, dyr).astype(f32)
    out = {"x": r.astype(f32), "y": np.zeros_like(r, dtype=f32), "dx": dxr.astype(f32), "dy": dyr,
           "dz": rays["dz"].astype(f32), "lambda_nm": rays["lambda_nm"].astype(f32)}
    return out, c, s, flip


def to_lab_frame(xo, yo, dxo, dyo, c, s, flip):
    """Inverse of canonical_frame for exit positions and directions (float64)."""
    c = np.asarray(c, np.float64)
    s = np.asarray(s, np.float64)
    sg = np.where(flip, -1.0, 1.0)
    yo, dyo = yo * sg, dyo * sg
    return c * xo - s * yo, s * xo + c * yo, c * dxo - s * dyo, s * dxo + c * dyo


def to_canonical_frame(xo, yo, dxo, dyo, c, s, flip):
    """Lab-frame exit positions and directions into the canonical frame."""
    c = np.asarray(c, np.float64)
    s = np.asarray(s, np.float64)
    sg = np.where(flip, -1.0, 1.0)
    return c * xo + s * yo, (c * yo - s * xo) * sg, c * dxo + s * dyo, (c * dyo - s * dxo) * sg


def features(rays: Dict[str, np.ndarray], p: MapParams) -> np.ndarray:
    if p.desc.canonical:
        rays = canonical_frame(rays)[0]
    x = np.stack([rays[k].astype(np.float64) for k in ("x", "y", "dx", "dy", "dz", "lambda_nm")], 1)
    return (x - p.in_shift) * p.in_scale


def act(z: np.ndarray, kind: int) -> np.ndarray:
    return np.tanh(z) if kind == ACT_TANH else np.maximum(z, 0.0)


def act_grad_from_output(h: np.ndarray, z: np.ndarray, kind: int) -> np.ndarray:
    return 1.0 - h * h if kind == ACT_TANH else (z > 0).astype(np.float64)


def forward(p: MapParams, xhat: np.ndarray):
    """FP64 forward.  Returns (o, cache) with o of shape (n, 6H)."""
    h = xhat
    hs, zs = [h], []
    L = len(p.W)
    for li in range(L):
        z = h @ p.W[li].T + p.b[li]
        zs.append(z)
        if li < L - 1:
            h = act(z, p.desc.activation)
            hs.append(h)
        else:
            h = z
    return h, (hs, zs)


def decode(o: np.ndarray, p: MapParams, rays: Dict[str, np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Head outputs (arrays of shape (H, n)) from raw network outputs; a
    canonical-input map needs the input rays to map its outputs back."""
    n = o.shape[0]
    H = p.desc.n_heads
    o = o.reshape(n, H, N_OUT).transpose(1, 0, 2)  # (H, n, 6)
    logit = o[..., 0]
    mask = logit > 0
    reg = p.out_shift[:, None, :] + p.out_scale[:, None, :] * o[..., 1:]
    x, y, dx, dy, thr = (reg[..., k] for k in range(5))
    if p.desc.canonical:
        if rays is None:
            raise ValueError("a canonical-input map needs the rays to decode")
        _, c, s, flip = canonical_frame(rays)
        x, y, dx, dy = to_lab_frame(x, y, dx, dy, c[None], s[None], flip[None])
    # the exit direction is a unit vector; its z component points toward
    # the object for a sensor-side map and toward the sensor for a forward one
    dz = (1.0 if p.desc.forward else -1.0) * np.sqrt(np.maximum(0.0, 1.0 - dx * dx - dy * dy))
    res = {"logit": logit, "mask": mask.astype(np.uint8)}
    for k, v in (("x", x), ("y", y), ("dx", dx), ("dy", dy), ("dz", dz)):
        res[k] = np.where(mask, v, np.nan)
    res["throughput"] = np.where(mask, thr, 0.0)
    return res


# ------------------------------------------------------------ rounding ----

def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even); returns float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out


def split_bf16(x: np.ndarray):
    hi = round_bf16(x)
    lo = round_bf16(np.asarray(x, np.float64) - hi)
    return hi, lo


FP8_MAX = 448.0


def round_fp8_e4m3(x: np.ndarray) -> np.ndarray:
    """OCP FP8 E4M3 (bias 7, 3 mantissa bits, max 448, subnormal step 2^-9),
    round to nearest even, saturating to +-448.  Returns float64."""
    x = np.asarray(x, np.float64)
    a = np.abs(x)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)                 # subnormals share the 2^-6 binade spacing
    step = np.exp2(e - 3.0)
    q = a / step
    r = np.floor(q)
    frac = q - r
    up = (frac > 0.5) | ((frac == 0.5) & (np.fmod(r, 2.0) == 1.0))
    r = r + up
    v = np.minimum(r * step, FP8_MAX)
    v = np.where(a > 0, v, 0.0)
    return np.copysign(v, x)


def pow2_scale(amax: float, target: float) -> float:
    """Largest power of two s with amax * s <= target (1 if amax == 0)."""
    if not (amax > 0) or not np.isfinite(amax):
        return 1.0
    s = 2.0 ** math.floor(math.log2(target / amax))
    while amax * s > target:
        s *= 0.5
    while amax * 2 * s <= target:
        s *= 2.0
    return float(s)


def fp8_layer_scales(p: MapParams):
    """Per hidden layer (1..depth-1): weight scale and activation scale used in
    FP8 mode.  Weights are scaled so max|W| maps to 448 or below, tanh
    activations (|h| <= 1) by 2^8."""
    ws, hs = [], []
    for li in range(1, len(p.W) - 1):
        ws.append(pow2_scale(float(np.abs(p.W[li]).max()), FP8_MAX))
        hs.append(256.0 if p.desc.activation == ACT_TANH else 1.0)
    return ws, hs


# The quantised network as the BF16 / FP8 kernels evaluate it, one rounding
# step per function.  The paper does not state the precision its networks
# run at; these rounding points are those of the reduced-precision kernels.
# A value passes through FP32 registers before it is rounded, so round_bf16
# rounds the FP32 value of its argument.

def input_layer_split(xhat: np.ndarray, W0: np.ndarray, b0: np.ndarray):
    """Input layer with inputs and weights split into BF16 hi + lo parts:
    z = x_hi W_hi + x_lo W_hi + x_hi W_lo + b (the x_lo W_lo term, below
    2^-16 of each product, is dropped).  Returns (z, (x_hi, x_lo))."""
    x_hi, x_lo = split_bf16(xhat)
    W_hi, W_lo = split_bf16(W0)
    return x_hi @ W_hi.T + x_lo @ W_hi.T + x_hi @ W_lo.T + b0, (x_hi, x_lo)


def output_layer_split(h: np.ndarray, Wo: np.ndarray, bo: np.ndarray) -> np.ndarray:
    """Output layer on BF16 activations with weights split into hi + lo:
    o = h W_hi + h W_lo + b."""
    W_hi, W_lo = split_bf16(Wo)
    return h @ W_hi.T + h @ W_lo.T + bo


def hidden_layer_bf16(h: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Pre-activation of a hidden layer: BF16 activations times BF16 weights,
    exact sums (the kernels accumulate in FP32)."""
    return h @ round_bf16(W).T + b


def transpose_weights_bf16(W: np.ndarray) -> np.ndarray:
    """The weights of the backward's transpose products (BF16)."""
    return round_bf16(W)


def activation_bf16(z: np.ndarray, kind: int) -> np.ndarray:
    """An activation rounded once to BF16."""
    return round_bf16(act(z, kind))


def hidden_layer_fp8(z_prev: np.ndarray, W: np.ndarray, b: np.ndarray, sw: float, sh: float,
                     kind: int) -> np.ndarray:
    """FP8 hidden layer: activations of the previous pre-activation rounded
    once to E4M3 after scaling by sh, weights rounded to E4M3 after scaling by
    sw, products summed exactly and divided by sw sh."""
    hq = round_fp8_e4m3(act(z_prev, kind) * sh)
    Wq = round_fp8_e4m3(W * sw)
    return (hq @ Wq.T) / (sw * sh) + b


# ----------------------------------------------- folded BF16 evaluation --
# tanh z = 1 - 2 r with r = 1 / (1 + 2^(k z)), k = 2 log2 e.  A layer
# z' = W h + b then reads z' = -2 W r + (b + W 1), and its scaled output
# u' = k z' feeds the next r = 1 / (1 + 2^u') directly.  The products with
# k are taken in FP32 (the packer's arithmetic) before any rounding.

K_TANH = float(np.float32(2.0 * math.log2(math.e)))


def scale_f32(a: np.ndarray, s: float) -> np.ndarray:
    """a * s as the packer computes it: FP32 operands, one FP32 rounding."""
    return (np.asarray(a, np.float32) * np.float32(s)).astype(np.float64)


def activation_folded_bf16(u: np.ndarray) -> np.ndarray:
    """r = 1 / (1 + 2^u) = (1 - tanh(u / k)) / 2, rounded once to BF16."""
    return round_bf16(1.0 / (1.0 + np.exp2(u)))


def hidden_layer_folded_bf16(r: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """u = Wq r + c with Wq = BF16(-2 k W) and c = k b - Wq 1 / 2, so that
    u = k (W' h + b) for h = 1 - 2 r and W' = Wq / (-2 k), the rounded weights
    (the sums exact; the kernels accumulate in FP32)."""
    Wq = round_bf16(scale_f32(W, -2.0 * K_TANH))
    c = scale_f32(b, K_TANH) - 0.5 * Wq.sum(1)
    return r @ Wq.T + c


def output_layer_folded(r: np.ndarray, Wo: np.ndarray, bo: np.ndarray) -> np.ndarray:
    """o = Wo (1 - 2 r) + bo with Wo split into BF16 hi + lo: the weights
    -2 W_hi and -2 W_lo (exact) and the bias bo + (W_hi + W_lo) 1."""
    W_hi, W_lo = split_bf16(Wo)
    return r @ (-2.0 * W_hi).T + r @ (-2.0 * W_lo).T + (bo + (W_hi + W_lo).sum(1))


def forward_folded_bf16(p: MapParams, xhat: np.ndarray) -> np.ndarray:
    """BF16 evaluation of a tanh map in the folded form: the split input layer
    on k W0 and k b0, hidden_layer_folded_bf16 between activations
    activation_folded_bf16, output_layer_folded."""
    L = len(p.W)
    u, _ = input_layer_split(xhat, scale_f32(p.W[0], K_TANH), scale_f32(p.b[0], K_TANH))
    r = activation_folded_bf16(u)
    for li in range(1, L - 1):
        r = activation_folded_bf16(hidden_layer_folded_bf16(r, p.W[li], p.b[li]))
    return output_layer_folded(r, p.W[L - 1], p.b[L - 1])


def forward_quantized(p: MapParams, xhat: np.ndarray, mode: str):
    """Forward pass with the kernels' rounding.  mode: "bf16" (BF16
    evaluation: forward_folded_bf16 for tanh maps, the unfolded form below for
    ReLU), "bf16_train" (the training forward: always unfolded) or "fp8".

    Unfolded bf16: split input layer, hidden layers with BF16 weights and
    BF16-rounded activations, split output layer.  fp8: the same input and
    output layers; every hidden layer is hidden_layer_fp8 (one FP8 rounding of
    each scaled activation); the last hidden activation is rounded to BF16."""
    if mode == "bf16" and p.desc.activation == ACT_TANH:
        return forward_folded_bf16(p, xhat)
    L = len(p.W)
    z, _ = input_layer_split(xhat, p.W[0], p.b[0])
    if mode == "fp8":
        ws, hsc = fp8_layer_scales(p)
        for li in range(1, L - 1):
            z = hidden_layer_fp8(z, p.W[li], p.b[li], ws[li - 1], hsc[li - 1], p.desc.activation)
        h = activation_bf16(z, p.desc.activation)
    else:
        h = activation_bf16(z, p.desc.activation)
        for li in range(1, L - 1):
            h = activation_bf16(hidden_layer_bf16(h, p.W[li], p.b[li]), p.desc.activation)
    return output_layer_split(h, p.W[L - 1], p.b[L - 1])


# ------------------------------------------------------------ training ----

def normalise_targets(t: Dict[str, np.ndarray], p: MapParams,
                      rays: Dict[str, np.ndarray] = None) -> np.ndarray:
    """(H, n, 5) normalised regression targets from per-head traced exit rays
    (for a canonical-input map first moved into each ray's canonical frame)."""
    t = {k: np.asarray(v, np.float64) for k, v in t.items()}
    if p.desc.canonical:
        _, c, s, flip = canonical_frame(rays)
        t["x"], t["y"], t["dx"], t["dy"] = to_canonical_frame(t["x"], t["y"], t["dx"], t["dy"],
                                                              c[None], s[None], flip[None])
    stk = np.stack([t[k] for k in ("x", "y", "dx", "dy", "throughput")], -1)  # (H, n, 5)
    return (stk - p.out_shift[:, None, :]) / p.out_scale[:, None, :]


def loss_and_grad(p: MapParams, xhat: np.ndarray, valid: np.ndarray, tnorm: np.ndarray,
                  w_bce: float = 1.0, w_l2: float = 1.0, w_cos: float = 0.0):
    """FP64 loss (total, bce, regression) and gradients (list of (dW, db)).

    valid: (H, n) 0/1; tnorm: (H, n, 5), ignored where valid == 0."""
    o, (hs, zs) = forward(p, xhat)
    losses, delta = loss_terms(p, o, valid, tnorm, w_bce, w_l2, w_cos)
    grads = [None] * len(p.W)
    for li in range(len(p.W) - 1, -1, -1):
        grads[li] = (delta.T @ hs[li], delta.sum(0))
        if li > 0:
            delta = (delta @ p.W[li]) * act_grad_from_output(hs[li], zs[li - 1], p.desc.activation)
    return losses, grads


@dataclasses.dataclass
class AdamState:
    m: np.ndarray
    v: np.ndarray
    step: int = 0


def adam_init(p: MapParams) -> AdamState:
    n = p.flat().size
    return AdamState(np.zeros(n), np.zeros(n), 0)


def grads_flat(grads) -> np.ndarray:
    return np.concatenate([np.concatenate([dW.reshape(-1), db.reshape(-1)]) for dW, db in grads])


def adam_step(p: MapParams, g: np.ndarray, st: AdamState, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    st.step += 1
    st.m = beta1 * st.m + (1 - beta1) * g
    st.v = beta2 * st.v + (1 - beta2) * g * g
    mhat = st.m / (1 - beta1 ** st.step)
    vhat = st.v / (1 - beta2 ** st.step)
    p.set_flat(p.flat() - lr * mhat / (np.sqrt(vhat) + eps))


def forward_quantized_cache(p: MapParams, xhat: np.ndarray):
    """BF16 forward of the training kernels, keeping what the backward uses:
    (o, (x_hi, x_lo, [h_1 .. h_depth]))."""
    L = len(p.W)
    z, (x_hi, x_lo) = input_layer_split(xhat, p.W[0], p.b[0])
    hs = [activation_bf16(z, p.desc.activation)]
    for li in range(1, L - 1):
        hs.append(activation_bf16(hidden_layer_bf16(hs[-1], p.W[li], p.b[li]), p.desc.activation))
    o = output_layer_split(hs[-1], p.W[L - 1], p.b[L - 1])
    return o, (x_hi, x_lo, hs)


def output_grad_split(d_out: np.ndarray) -> np.ndarray:
    """The output gradient as the backward kernels carry it: BF16 hi + lo."""
    d_hi, d_lo = split_bf16(d_out)
    return d_hi + d_lo


def hidden_grad_bf16(delta: np.ndarray, h: np.ndarray, kind: int) -> np.ndarray:
    """Gradient of a hidden pre-activation: the incoming gradient times the
    activation derivative taken from the stored BF16 activation (1 - h^2 for
    tanh, [h > 0] for ReLU), rounded once to BF16."""
    dphi = 1.0 - h * h if kind == ACT_TANH else (h > 0).astype(np.float64)
    return round_bf16(delta * dphi)


def backward_quantized(p: MapParams, cache, d_out: np.ndarray):
    """Parameter gradient for a given output gradient d_out (n, 6H), with the
    training kernels' rounding: the output gradient enters split into BF16
    hi + lo (against BF16 output weights for the transpose product); every
    hidden-layer gradient is hidden_grad_bf16, then used in BF16 for its
    weight gradient (against the stored BF16 activations, or the split
    inputs for the first layer), for its bias gradient (sum over rays) and
    for the next transpose product (against BF16 weights).  Sums are exact
    here (FP64); the kernels accumulate in FP32."""
    x_hi, x_lo, hs = cache
    L = len(p.W)
    d = output_grad_split(d_out)
    grads = [None] * L
    grads[L - 1] = (d.T @ hs[-1], d.sum(0))
    delta = d @ transpose_weights_bf16(p.W[L - 1])
    for li in range(L - 2, -1, -1):
        delta_b = hidden_grad_bf16(delta, hs[li], p.desc.activation)
        if li == 0:
            grads[0] = (delta_b.T @ (x_hi + x_lo), delta_b.sum(0))
        else:
            grads[li] = (delta_b.T @ hs[li - 1], delta_b.sum(0))
            delta = delta_b @ transpose_weights_bf16(p.W[li])
    return grads


COS_EPS = 1e-6   # floor of 1 - dx^2 - dy^2 under the square root of the direction loss


def _dir3(dx, dy):
    """Unit-sphere direction toward the object from (dx, dy): dz = -sqrt(s),
    s = max(COS_EPS, 1 - dx^2 - dy^2); also returns s and whether s was
    floored."""
    s = 1.0 - dx * dx - dy * dy
    floored = s < COS_EPS
    s = np.where(floored, COS_EPS, s)
    return -np.sqrt(s), s, floored


def loss_terms(p: MapParams, o: np.ndarray, valid: np.ndarray, tnorm: np.ndarray,
               w_bce: float = 1.0, w_l2: float = 1.0, w_cos: float = 0.0):
    """Loss (total, bce, regression) and its gradient with respect to o (n, 6H).

    Regression part, on rays whose target is valid:
      w_cos == 0: w_l2 * mean squared error of the five normalised outputs;
      w_cos > 0:  w_l2 * mean squared error of x, y, throughput (normalised)
                  + w_cos * mean (1 - cos angle) between predicted and target
                  exit directions (Sec. 5.1 trains directions with a cosine
                  similarity loss); a direction is (dx, dy, -sqrt(1 - dx^2 -
                  dy^2)) in lens units, the square root's argument floored
                  at COS_EPS."""
    n = o.shape[0]
    H = p.desc.n_heads
    oo = o.reshape(n, H, N_OUT).transpose(1, 0, 2)
    logit = oo[..., 0]
    v = valid.astype(np.float64)
    on = v[..., None] > 0
    bce = np.maximum(logit, 0) - logit * v + np.log1p(np.exp(-np.abs(logit)))
    sig = 1.0 / (1.0 + np.exp(-logit))
    t = np.where(on, tnorm, 0.0)
    diff = np.where(on, oo[..., 1:] - t, 0.0)
    g = np.zeros_like(oo)
    l_bce = w_bce * bce.sum() / (n * H)
    g[..., 0] = w_bce * (sig - v) / (n * H)
    if w_cos == 0.0:
        l_reg = w_l2 * (diff * diff).sum() / (5 * n * H)
        g[..., 1:] = w_l2 * 2.0 * diff / (5 * n * H)
    else:
        pos = [0, 1, 4]   # x, y, throughput among the five regression outputs
        l_reg = w_l2 * (diff[..., pos] ** 2).sum() / (3 * n * H)
        for k in pos:
            g[..., 1 + k] = w_l2 * 2.0 * diff[..., k] / (3 * n * H)
        sh, sc = p.out_shift[:, None, :], p.out_scale[:, None, :]
        dxp = sh[..., 2] + sc[..., 2] * oo[..., 3]
        dyp = sh[..., 3] + sc[..., 3] * oo[..., 4]
        dxt = sh[..., 2] + sc[..., 2] * t[..., 2]
        dyt = sh[..., 3] + sc[..., 3] * t[..., 3]
        dzp, sp, flp = _dir3(dxp, dyp)
        dzt, _, _ = _dir3(dxt, dyt)
        nt = np.sqrt(dxt * dxt + dyt * dyt + dzt * dzt)
        qx, qy, qz = dxt / nt, dyt / nt, dzt / nt
        nu = np.sqrt(dxp * dxp + dyp * dyp + dzp * dzp)
        dot = dxp * qx + dyp * qy + dzp * qz
        cosv = dot / nu
        l_reg += w_cos * np.where(v > 0, 1.0 - cosv, 0.0).sum() / (n * H)
        # d cos / d u = q / |u| - (u . q) u / |u|^3, and d dz / d(dx, dy) =
        # (dx, dy) / sqrt(s) unless s was floored
        gx = qx / nu - dot * dxp / nu ** 3
        gy = qy / nu - dot * dyp / nu ** 3
        gz = qz / nu - dot * dzp / nu ** 3
        dzdx = np.where(flp, 0.0, dxp / np.sqrt(sp))
        dzdy = np.where(flp, 0.0, dyp / np.sqrt(sp))
        scale = -w_cos * v / (n * H)
        g[..., 3] = scale * (gx + gz * dzdx) * sc[..., 2]
        g[..., 4] = scale * (gy + gz * dzdy) * sc[..., 3]
    return (l_bce + l_reg, l_bce, l_reg), g.transpose(1, 0, 2).reshape(n, H * N_OUT)


def loss_and_grad_quantized(p: MapParams, xhat: np.ndarray, valid: np.ndarray, tnorm: np.ndarray,
                            w_bce: float = 1.0, w_l2: float = 1.0, w_cos: float = 0.0):
    """Loss and parameter gradient of one training step with the kernels'
    rounding (forward_quantized_cache, loss_terms, backward_quantized)."""
    o, cache = forward_quantized_cache(p, xhat)
    losses, d_out = loss_terms(p, o, valid, tnorm, w_bce, w_l2, w_cos)
    return losses, backward_quantized(p, cache, d_out)
