"""Host twin of the counter-based ray generator (synth.philox_rays):
Philox4x64-10 pinned to numpy's own Philox bit generator, and the ray
distribution checked against its definition."""
import numpy as np

import synth


def test_philox_matches_numpy():
    """numpy's Philox is Philox4x64-10; it increments its 256-bit counter
    before each block, so block c of numpy (started at counter 0) is counter
    c + 1 here."""
    rng = np.random.default_rng(3)
    for key in [(0, 0), (5, 7), (2 ** 64 - 1, 2 ** 63 + 11)]:
        for start in [0, 123456789, 2 ** 63 + 5]:
            bg = np.random.Philox(key=np.array(key, np.uint64),
                                  counter=np.array([start, 0, 0, 0], np.uint64))
            raw = bg.random_raw(4 * 16).reshape(16, 4)
            ctr = (np.arange(16, dtype=np.uint64) + np.uint64(start) + np.uint64(1))
            z = np.zeros(16, np.uint64)
            got = np.stack(synth.philox4x64_10((ctr, z, z, z), key), 1)
            assert np.array_equal(got, raw), (key, start)
    # a counter with every word set (carry paths of the multiply)
    c = [np.array([2 ** 64 - 1], np.uint64)] * 4
    bg = np.random.Philox(key=np.array([9, 9], np.uint64),
                          counter=np.array([2 ** 64 - 2] + [2 ** 64 - 1] * 3, np.uint64))
    assert np.array_equal(np.stack(synth.philox4x64_10(c, (9, 9)), 1)[0], bg.random_raw(4))
    del rng


def test_ray_distribution():
    L = synth.config_lens(2)
    n = 200000
    r = synth.philox_rays(L, n, seed=77)
    assert all(v.dtype == np.float32 and v.shape == (n,) for v in r.values())
    assert r["x"].min() >= -18 and r["x"].max() < 18 and r["y"].min() >= -12 and r["y"].max() < 12
    assert r["lambda_nm"].min() >= 400 and r["lambda_nm"].max() < 700
    d = np.stack([r["dx"], r["dy"], r["dz"]], 1).astype(np.float64)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=2e-7) and np.all(d[:, 2] < 0)
    # back-project to the rear vertex plane: inside the clear-aperture disk,
    # uniform by area (mean of rho^2 / sd^2 = 1/2)
    rear = L.surfaces[-1]
    t = rear.thickness / -d[:, 2]
    px = r["x"] + t * d[:, 0]
    py = r["y"] + t * d[:, 1]
    q = (px ** 2 + py ** 2) / rear.semi_diameter ** 2
    assert q.max() <= 1 + 1e-5
    assert abs(q.mean() - 0.5) < 5e-3
    for k, (lo, hi) in (("x", (-18, 18)), ("y", (-12, 12)), ("lambda_nm", (400, 700))):
        assert abs(r[k].mean() - (lo + hi) / 2) < 0.01 * (hi - lo)


def test_counter_slices_are_independent():
    L = synth.config_lens(1)
    a = synth.philox_rays(L, 1000, seed=5)
    b = synth.philox_rays(L, 300, seed=5, first=600)
    for k in a:
        assert np.array_equal(a[k][600:900], b[k])
    c = synth.philox_rays(L, 1000, seed=6)
    assert not np.array_equal(a["x"], c["x"])
