"""Symmetry-reduced map input (oracle/mlp.py canonical_frame, to_lab_frame,
to_canonical_frame), pinned by the invariances Sec. 4.1 states and by the
FP64 tracer oracle: the lens commutes with rotations about the axis and with
mirrors through it, so tracing the canonical ray and mapping the exit ray
back must reproduce the trace of the original ray."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp


def rotate(rays, theta, mirror=False):
    """Rotate (and optionally mirror y -> -y first) sensor points and
    directions in float64, rounded to float32."""
    f = np.float32
    x, y = rays["x"].astype(np.float64), rays["y"].astype(np.float64)
    dx, dy = rays["dx"].astype(np.float64), rays["dy"].astype(np.float64)
    if mirror:
        y, dy = -y, -dy
    c, s = np.cos(theta), np.sin(theta)
    out = dict(rays)
    out["x"], out["y"] = (c * x - s * y).astype(f), (s * x + c * y).astype(f)
    out["dx"], out["dy"] = (c * dx - s * dy).astype(f), (s * dx + c * dy).astype(f)
    return out


def test_canonical_domain():
    rays = synth.config_rays(2, 20000)
    can, c, s, flip = mlp.canonical_frame(rays)
    assert np.all(can["y"] == 0) and np.all(can["x"] >= 0) and np.all(can["dy"] >= 0)
    assert np.array_equal(can["dz"], rays["dz"]) and np.array_equal(can["lambda_nm"], rays["lambda_nm"])
    r = np.hypot(rays["x"].astype(np.float64), rays["y"].astype(np.float64))
    assert np.allclose(can["x"], r, rtol=2e-7)
    n0 = np.hypot(rays["dx"].astype(np.float64), rays["dy"].astype(np.float64))
    n1 = np.hypot(can["dx"].astype(np.float64), can["dy"].astype(np.float64))
    assert np.allclose(n0, n1, atol=3e-7)
    assert np.allclose(c.astype(np.float64) ** 2 + s.astype(np.float64) ** 2, 1.0, atol=3e-7)
    assert 0.3 < flip.mean() < 0.7


def test_special_points():
    f = np.float32
    rays = {"x": np.array([0, -3, 0, 5], f), "y": np.array([0, 0, 2, 0], f),
            "dx": np.array([0.1, 0.1, 0.1, 0.1], f), "dy": np.array([0.2, 0.2, 0.2, -0.2], f),
            "dz": np.full(4, -0.9, f), "lambda_nm": np.full(4, 500, f)}
    can, c, s, flip = mlp.canonical_frame(rays)
    assert (c[0], s[0], flip[0]) == (1, 0, False)          # on the axis: identity
    assert (c[1], s[1]) == (-1, 0) and can["x"][1] == 3     # rotation by pi
    assert (c[2], s[2]) == (0, 1) and can["x"][2] == 2      # rotation by pi/2
    assert can["dx"][2] == f(0.2) and can["dy"][2] == f(0.1) and flip[2]
    assert flip[3] and can["dy"][3] == f(0.2)               # mirror only


def test_round_trip():
    rng = np.random.default_rng(0)
    v = rng.normal(size=(4, 1000))
    theta = rng.uniform(0, 7, 1000)
    c, s = np.cos(theta), np.sin(theta)
    flip = rng.integers(0, 2, 1000).astype(bool)
    back = mlp.to_lab_frame(*mlp.to_canonical_frame(*v, c, s, flip), c, s, flip)
    assert np.allclose(np.array(back), v, atol=1e-12)


@pytest.mark.parametrize("theta,mirror", [(0.7, False), (2.9, True), (-1.3, False), (np.pi, True)])
def test_canonical_input_is_invariant(theta, mirror):
    rays = synth.config_rays(2, 5000)
    a = mlp.canonical_frame(rays)[0]
    b = mlp.canonical_frame(rotate(rays, theta, mirror))[0]
    for k in ("x", "dx", "dy"):
        assert np.allclose(a[k], b[k], atol=2e-5), k


def test_tracer_commutes_with_canonical_frame():
    """to_lab_frame(trace(canonical ray)) == trace(ray) for transmit and a
    ghost: fixes the sense of the rotation and of the mirror."""
    L = synth.config_lens(2)
    rays = synth.config_rays(2, 20000)
    can, c, s, flip = mlp.canonical_frame(rays)
    for path in [(0, 0, 0), (1, 3, 8)]:
        a = oracle.trace(L, rays, path)
        b = oracle.trace(L, can, path)
        both = (a["mask"] == 1) & (b["mask"] == 1)
        assert both.sum() > 300
        assert np.mean(a["mask"] == b["mask"]) > 0.999
        X, Y, DX, DY = mlp.to_lab_frame(b["x"], b["y"], b["dx"], b["dy"], c, s, flip)
        assert np.abs(X - a["x"])[both].max() < 2e-3
        assert np.abs(Y - a["y"])[both].max() < 2e-3
        assert np.abs(DX - a["dx"])[both].max() < 1e-4
        assert np.abs(DY - a["dy"])[both].max() < 1e-4
        assert np.abs(b["throughput"] - a["throughput"])[both].max() < 1e-5


def test_canonical_map_is_equivariant():
    """Any parameters: the canonical-input network maps rotated/mirrored
    inputs to rotated/mirrored outputs (up to the float32 canonicalisation)."""
    rays = synth.config_rays(2, 3000)
    desc = mlp.MapDesc(32, 3, 2, mlp.ACT_TANH, canonical=True)
    p = mlp.init_params(desc, 3)
    rng = np.random.default_rng(1)
    for b in p.b:
        b[:] = rng.normal(0, 0.3, b.shape)
    p.in_scale = np.array([0.1, 0.1, 3, 3, 3, 0.01])
    p.in_shift = np.array([10, 0, 0, 0, -0.9, 550])
    p.out_scale = rng.uniform(1, 5, (2, 5))
    for theta, mirror in [(0.4, False), (-2.0, True)]:
        rr = rotate(rays, theta, mirror)
        d0 = mlp.decode(mlp.forward(p, mlp.features(rays, p))[0], p, rays)
        d1 = mlp.decode(mlp.forward(p, mlp.features(rr, p))[0], p, rr)
        # expected: the outputs of d0 moved by the same mirror + rotation
        ex, ey = d0["x"], d0["y"]
        edx, edy = d0["dx"], d0["dy"]
        if mirror:
            ey, edy = -ey, -edy
        cth, sth = np.cos(theta), np.sin(theta)
        ok = (d0["mask"] == 1) & (d1["mask"] == 1)
        assert np.mean(d0["mask"] == d1["mask"]) > 0.995
        assert np.allclose((cth * ex - sth * ey)[ok], d1["x"][ok], atol=5e-4)
        assert np.allclose((sth * ex + cth * ey)[ok], d1["y"][ok], atol=5e-4)
        assert np.allclose((cth * edx - sth * edy)[ok], d1["dx"][ok], atol=5e-4)
        assert np.allclose(d0["throughput"][ok], d1["throughput"][ok], atol=5e-4)


def test_canonical_targets_round_trip():
    """normalise_targets in the canonical frame, then decode of the exact
    normalised targets as outputs, gives the lab-frame targets back."""
    rays = synth.config_rays(2, 2000)
    L = synth.config_lens(2)
    t = oracle.trace(L, rays)
    ok = t["mask"] == 1
    desc = mlp.MapDesc(32, 2, 1, mlp.ACT_TANH, canonical=True)
    p = mlp.init_params(desc, 0)
    p.out_shift = np.array([[1.0, -2.0, 0.01, 0.02, 0.5]])
    p.out_scale = np.array([[3.0, 4.0, 0.1, 0.2, 0.3]])
    tn = mlp.normalise_targets({k: t[k][None] for k in ("x", "y", "dx", "dy", "throughput")}, p, rays)
    o = np.zeros((2000, 6))
    o[:, 0] = 1.0
    o[:, 1:] = np.nan_to_num(tn[0])
    d = mlp.decode(o, p, rays)
    for k in ("x", "y", "dx", "dy", "throughput"):
        assert np.allclose(d[k][0][ok], t[k][ok], atol=1e-9), k
