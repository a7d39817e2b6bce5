"""The benchmark states the map's exit-ray error against the FP32 GPU
tracer.  On a fitted map, that error and the error against the FP64 oracle
agree to the tracer's own bound (1e-5 mm, 1e-6 rad, 1e-5 throughput): every
order statistic of per-ray errors moves by at most the per-ray bound, and
masks differ only for rays in the aperture-edge band."""
import numpy as np
import pytest

import oracle
import synth
from paper_2605_04017_amd import fit as F

pytestmark = pytest.mark.gpu


def test_map_error_against_tracer_equals_error_against_oracle():
    import torch
    import paper_2605_04017_amd as lt
    import bench
    dev = torch.device("cuda:0")
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    pool_np = synth.make_rays(lens, 1 << 20, 3002)
    pool = {k: torch.from_numpy(v).to(dev) for k, v in pool_np.items()}
    ex = lt.lt_trace(h, (0, 0, 0), pool)
    ok = ex["mask"].bool()
    reg = torch.stack([ex[k][ok] for k in ("x", "y", "dx", "dy", "throughput")], 1).double().cpu().numpy()
    norms = F.map_norms(pool_np, [(ok.cpu().numpy(), reg)])
    m = lt.lt_map_create(128, 5, 1)
    lt.lt_map_set_params(m, torch.from_numpy(F.init_params(128, 5, 1, 5)).to(dev))
    lt.lt_map_set_norm(m, norms[0], norms[1], norms[2].reshape(-1), norms[3].reshape(-1))
    batch = 65536
    ws = lt.workspace(m, batch)
    for k in range(1, 401):
        lo = ((k - 1) * batch) % ((1 << 20) - batch + 1)
        rb = {f: v[lo:lo + batch] for f, v in pool.items()}
        tb = {"valid": ex["mask"][lo:lo + batch].reshape(1, -1)}
        for f in ("x", "y", "dx", "dy", "throughput"):
            tb[f] = ex[f][lo:lo + batch].reshape(1, -1)
        lt.lt_map_train_step(m, rb, tb, {"lr": 2e-3 * 0.5 ** (k / 100), "step": k, "w_bce": 1.0,
                                         "w_l2": 4.0}, ws)
    n = 32768
    rays_np = synth.config_rays(2, n)
    rays = {k: torch.from_numpy(v).to(dev) for k, v in rays_np.items()}
    for dt in (lt.LT_F32, lt.LT_BF16):
        vs_tracer = bench.map_error(lt, h, m, dt, rays, n)
        g = bench.eval_host(lt.lt_map_eval(m, dt, rays))
        torch.cuda.synchronize()
        vs_oracle = bench.exit_error(g, oracle.trace(lens, rays_np), n)
        assert abs(vs_tracer["mask_agreement"] - vs_oracle["mask_agreement"]) <= 1e-3
        for k, bound in (("pos_mm_p50", 1e-5), ("pos_mm_p99", 1e-5), ("dir_rad_p50", 1e-6),
                         ("dir_rad_p99", 1e-6), ("throughput_abs_p99", 1e-5)):
            assert abs(vs_tracer[k] - vs_oracle[k]) <= bound + 1e-7, (dt, k, vs_tracer[k], vs_oracle[k])
        print(f"[map error] dtype {dt}: position p50 {vs_tracer['pos_mm_p50']:.4f} mm against the "
              f"tracer, {vs_oracle['pos_mm_p50']:.4f} mm against the oracle", flush=True)
