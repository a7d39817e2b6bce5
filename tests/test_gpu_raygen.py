"""Device ray generator (lt_rays_generate) against its host twin
(synth.philox_rays): the Philox words must agree exactly, which shows up as
bit-identical sensor points and wavelengths (single FP32 roundings of exact
values on both sides); directions go through FP32 sqrt, sincos and a
normalisation on the device and FP64 on the host, so they agree to a few
FP32 ulps (bound 1e-6)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.mark.parametrize("cfg,n,seed,first", [(2, 1 << 20, 17, 0), (1, 1001, 3, 2 ** 40 + 7),
                                              (5, 4097, 2 ** 64 - 1, 2 ** 64 - 100)])
def test_device_rays_match_host_twin(dev, cfg, n, seed, first):
    import torch
    import paper_2605_04017_amd as lt
    L = synth.serve_lenses()[3] if cfg == 5 else synth.config_lens(cfg)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    got = {k: v.cpu().numpy() for k, v in lt.lt_rays_generate(h, n, seed, first).items()}
    torch.cuda.synchronize()
    with np.errstate(over="ignore"):
        ref = synth.philox_rays(L, n, seed, first)
    for k in ("x", "y", "lambda_nm"):
        assert np.array_equal(got[k], ref[k]), k
    for k in ("dx", "dy", "dz"):
        err = np.abs(got[k].astype(np.float64) - ref[k])
        assert err.max() <= 1e-6, (k, err.max())
    print(f"[raygen] cfg {cfg} n {n}: direction max diff "
          f"{max(np.abs(got[k].astype(np.float64) - ref[k]).max() for k in ('dx', 'dy', 'dz')):.2e}",
          flush=True)


def test_device_counter_slices(dev):
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    a = lt.lt_rays_generate(h, 3000, 9)
    b = lt.lt_rays_generate(h, 1000, 9, first=1000)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k][1000:2000], b[k])
    lt.lt_rays_generate(h, 0, 9)   # n = 0 is a no-op
    with pytest.raises(lt.LtError):
        lt.lt_rays_generate(h, 10, 9, half_width=-1.0)


def test_generated_rays_trace_like_host_rays(dev):
    """Rays drawn on the device have the workload's transmit valid fraction."""
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    n = 1 << 20
    r = lt.lt_rays_generate(h, n, 4242)
    ex = lt.lt_trace(h, (0, 0, 0), r)
    host = {k: torch.from_numpy(v).to(dev) for k, v in synth.config_rays(2, n).items()}
    ex2 = lt.lt_trace(h, (0, 0, 0), host)
    torch.cuda.synchronize()
    f1 = float(ex["mask"].float().mean())
    f2 = float(ex2["mask"].float().mean())
    assert abs(f1 - f2) < 3e-3, (f1, f2)
