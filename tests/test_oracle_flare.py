"""Pins of the oracle's sensor-image formation (forward light tracing,
Sec. 3: each valid exit ray adds I * dot(w_out, n_cmos) to its pixel under a
box filter), checked against facts fixed by the definition's geometry:
pixel centres, frame edges, energy conservation, mirror symmetry, and a
physical image of a point light on the axis."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import flare

SENSOR = (36.0, 24.0, 480, 320)


def _centres(sensor):
    w, h, nx, ny = sensor
    xc = -w / 2 + (np.arange(nx) + 0.5) * (w / nx)
    yc = -h / 2 + (np.arange(ny) + 0.5) * (h / ny)
    return xc, yc


def test_pixel_centres_land_in_their_pixel():
    for sensor in (SENSOR, (36.0, 24.0, 7, 5), (10.0, 10.0, 1, 1), (24.0, 24.0, 1000, 3)):
        xc, yc = _centres(sensor)
        X, Y = np.meshgrid(xc, yc)
        inside, ix, iy = flare.pixel_of(X.ravel(), Y.ravel(), sensor)
        assert inside.all()
        assert np.array_equal(ix, np.tile(np.arange(sensor[2]), sensor[3]))
        assert np.array_equal(iy, np.repeat(np.arange(sensor[3]), sensor[2]))


def test_frame_edges():
    w, h, nx, ny = SENSOR
    f = np.float32
    # (the last FP32 value below the right edge may round onto it in pixel
    # units, so the inside probe sits 1e-4 mm in)
    x = np.array([-w / 2, w / 2, np.nextafter(f(-w / 2), f(-100)), w / 2 - 1e-4, 0.0,
                  np.nan, 0.0], np.float32)
    y = np.array([0.0, 0.0, 0.0, 0.0, h / 2, 0.0, np.inf], np.float32)
    inside, ix, iy = flare.pixel_of(x, y, SENSOR)
    # the frame is half open: the left edge belongs to pixel 0, the right edge is outside
    assert inside.tolist() == [True, False, False, True, False, False, False]
    assert ix[0] == 0 and ix[3] == nx - 1
    assert iy[0] == ny // 2


def test_uniform_grid_gives_flat_image():
    xc, yc = _centres(SENSOR)
    X, Y = np.meshgrid(xc, yc)
    n = X.size
    img = flare.splat(X.ravel(), Y.ravel(), np.ones(n), np.ones(n), SENSOR)
    assert img.shape == (1, SENSOR[3], SENSOR[2])
    assert np.array_equal(img[0], np.ones((SENSOR[3], SENSOR[2])))


def test_energy_conservation_and_masking():
    rng = np.random.default_rng(3)
    n = 20000
    x = rng.uniform(-30, 30, n).astype(np.float32)
    y = rng.uniform(-20, 20, n).astype(np.float32)
    dz = rng.uniform(0.5, 1.0, n)
    thr = rng.uniform(0.0, 1.0, n)
    mask = rng.uniform(size=n) < 0.7
    img = flare.splat(x, y, dz, thr, SENSOR, mask=mask, scale=0.25)
    w, h = SENSOR[:2]
    on = mask & (np.abs(x) < w / 2) & (np.abs(y) < h / 2)
    assert math.isclose(img.sum(), 0.25 * (thr[on] * dz[on]).sum(), rel_tol=1e-12)
    # NaN positions never land
    x2 = x.copy()
    x2[::2] = np.nan
    img2 = flare.splat(x2, y, dz, thr, SENSOR, mask=mask)
    on2 = on.copy()
    on2[::2] = False
    assert math.isclose(img2.sum(), (thr[on2] * dz[on2]).sum(), rel_tol=1e-12)


def test_mirror_symmetry():
    """x -> -x mirrors the image left-right (rays away from pixel edges)."""
    rng = np.random.default_rng(4)
    w, h, nx, ny = SENSOR
    ix = rng.integers(0, nx, 5000)
    iy = rng.integers(0, ny, 5000)
    fx = rng.uniform(0.1, 0.9, 5000)
    fy = rng.uniform(0.1, 0.9, 5000)
    x = -w / 2 + (ix + fx) * (w / nx)
    y = -h / 2 + (iy + fy) * (h / ny)
    wt = rng.uniform(size=5000)
    a = flare.splat(x, y, np.ones(5000), wt, SENSOR)[0]
    b = flare.splat(-x, y, np.ones(5000), wt, SENSOR)[0]
    assert np.allclose(a[:, ::-1], b, rtol=0, atol=1e-12)


def test_images_per_path_sum_to_the_single_image():
    rng = np.random.default_rng(5)
    n, p = 3000, 4
    x = rng.uniform(-20, 20, n * p)
    y = rng.uniform(-14, 14, n * p)
    wt = rng.uniform(size=n * p)
    per = flare.splat(x, y, np.ones(n * p), wt, SENSOR, n_per_image=n)
    one = flare.splat(x, y, np.ones(n * p), wt, SENSOR)
    assert per.shape[0] == p
    assert np.allclose(per.sum(0), one[0], rtol=0, atol=1e-12)
    for k in range(p):
        sl = slice(k * n, (k + 1) * n)
        assert np.allclose(per[k], flare.splat(x[sl], y[sl], np.ones(n), wt[sl], SENSOR)[0])


def test_on_axis_point_light_image():
    """A point light at infinity on the axis, traced forward through the
    11-surface lens (sensor at the paraxial focus): the transmit image is
    centred on the axis (rotational symmetry), concentrated in a small blur
    spot, and carries at most the energy that entered (I <= 1, dz <= 1)."""
    L = synth.config_lens(2)
    n = 40000
    rays = synth.make_forward_rays(L, n, 21, direction=(0.0, 0.0, 1.0), aperture_scale=1.0,
                                   lam_range=(550.0, 550.0))
    sensor = (2.0, 2.0, 200, 200)
    img = flare.render_forward(L, rays, [(0, 0, 0)], sensor)[(0, 0, 0)]
    t = oracle.trace(L, rays, (0, 0, 0), forward=True)
    ok = t["mask"] == 1
    assert ok.sum() > n // 20
    # every valid ray of the on-axis beam lands within 1 mm of the axis
    assert np.abs(t["x"][ok]).max() < 1.0 and np.abs(t["y"][ok]).max() < 1.0
    tot = img.sum()
    assert math.isclose(tot, (t["throughput"][ok] * t["dz"][ok]).sum(), rel_tol=1e-12)
    assert tot <= ok.sum()
    yy, xx = np.mgrid[0:200, 0:200]
    cx = ((xx + 0.5) * img).sum() / tot * 0.01 - 1.0
    cy = ((yy + 0.5) * img).sum() / tot * 0.01 - 1.0
    assert abs(cx) < 5e-3 and abs(cy) < 5e-3
    # the four quadrants carry the same energy to sampling noise
    q = [img[:100, :100].sum(), img[:100, 100:].sum(), img[100:, :100].sum(), img[100:, 100:].sum()]
    assert max(q) / min(q) < 1.1


@pytest.mark.parametrize("theta_deg", [5.0, 10.0])
def test_off_axis_point_light_image_height(theta_deg):
    """The transmit image of a distant off-axis point light sits near the
    paraxial image height EFL * tan(theta) (the lens is close to
    distortion-free at these angles; 3 % allowed)."""
    L = synth.config_lens(2)
    th = math.radians(theta_deg)
    n = 30000
    rays = synth.make_forward_rays(L, n, 22, direction=(math.sin(th), 0.0, math.cos(th)),
                                   aperture_scale=1.0, lam_range=(550.0, 550.0))
    t = oracle.trace(L, rays, (0, 0, 0), forward=True)
    ok = t["mask"] == 1
    assert ok.sum() > 200
    wgt = t["throughput"][ok] * t["dz"][ok]
    xc = (t["x"][ok] * wgt).sum() / wgt.sum()
    yc = (t["y"][ok] * wgt).sum() / wgt.sum()
    h = 50.0 * math.tan(th)   # EFL 50 mm by construction (paraxial design of the input generator)
    # the beam travels toward +x (the source lies at -x): the image is
    # inverted, on the +x side
    assert abs(xc - h) < 0.03 * h
    assert abs(yc) < 1e-3 * h + 1e-3
