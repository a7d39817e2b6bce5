"""The paper's training-data recipe (Sec. 5.1 "Data Collection") as the
library draws it: Markov-chain rays for the regressor that are all valid
and whose exits are the tracer's, a balanced classifier set whose invalid
half is invalid, CIE-weighted wavelengths; and the epoch loop's schedule."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def test_sampler_dataset(dev):
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd import fit as F
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    path = (1, 2, 10)
    n = 50000
    d = F.sampler_dataset(h, path, n, 11, n_chains=1 << 14, burn_in=64, thin=4)
    torch.cuda.synchronize()
    # regressor rays: every one valid, exits exactly the tracer's
    t = lt.lt_trace(h, path, d["reg_rays"])
    torch.cuda.synchronize()
    assert int(t["mask"].sum()) == n
    for k in F.REG_FIELDS:
        assert torch.equal(t[k].view(torch.int32), d["reg_exit"][k].view(torch.int32)), k
    # classifier set: balanced, labels equal the tracer's validity
    assert d["cls_valid"].numel() == 2 * n and int(d["cls_valid"].sum()) == n
    tc = lt.lt_trace(h, path, d["cls_rays"])
    torch.cuda.synchronize()
    assert torch.equal(tc["mask"], d["cls_valid"])
    # wavelengths: CIE-weighted.  The invalid half is nearly the unconditioned
    # draw (98 % of rays miss this ghost): its mass in 500-600 nm against the
    # oracle's CIE distribution (0.418; a uniform draw gives 1/3)
    from oracle import sampling as S
    lam = d["cls_rays"]["lambda_nm"][d["cls_valid"] == 0].cpu().numpy()
    assert lam.min() >= 400 and lam.max() <= 700
    c = lambda x: float(S.cie_cdf(np.array([x]))[0])
    want = (c(600) - c(500)) / (c(700) - c(400))
    got = float(np.mean((lam > 500) & (lam < 600)))
    assert abs(got - want) < 0.02, (got, want)


def test_fit_epochs_reduces_loss(dev):
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd import fit as F
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    rays = lt.lt_rays_generate(h, 1 << 15, 5)
    ex = lt.lt_trace(h, (0, 0, 0), rays)
    rays_np = {k: v.cpu().numpy() for k, v in rays.items()}
    ok = ex["mask"].bool()
    reg = torch.stack([ex[k][ok] for k in F.REG_FIELDS], 1).double().cpu().numpy()
    norms = F.map_norms(rays_np, [(ok.cpu().numpy(), reg)])
    m = lt.lt_map_create(32, 2, 1, lt.LT_ACT_TANH)
    lt.lt_map_set_params(m, torch.from_numpy(F.init_params(32, 2, 1, 3)).to(dev))
    lt.lt_map_set_norm(m, norms[0], norms[1], norms[2].reshape(-1), norms[3].reshape(-1))
    tg = {"valid": ex["mask"].reshape(1, -1)}
    for k in F.REG_FIELDS:
        tg[k] = ex[k].reshape(1, -1)
    cfg = {"w_bce": 1.0, "w_l2": 1.0}
    s1, l1 = F.fit_epochs(m, rays, tg, 1, 4096, cfg, 7, lr=lambda k: 1e-3)
    s2, l2 = F.fit_epochs(m, rays, tg, 4, 4096, cfg, 8, lr=lambda k: 1e-3)
    torch.cuda.synchronize()
    assert s1 == 8 and s2 == 32
    assert float(l2[0]) < float(l1[0])


def test_fit_epochs_graph_runs_match_eager(dev):
    """fit_epochs with recorded runs (graph_steps = 3 of the 8 steps per
    epoch: two replayed runs and two eager steps each epoch) leaves exactly
    the parameters of the eager loop after two epochs."""
    import torch
    import paper_2605_04017_amd as lt
    from paper_2605_04017_amd import fit as F
    lens = synth.config_lens(2)
    h = lt.lt_lens_create(lens.surfaces, lens.glasses)
    rays = lt.lt_rays_generate(h, 1 << 15, 15)
    ex = lt.lt_trace(h, (0, 0, 0), rays)
    tg = {"valid": ex["mask"].reshape(1, -1)}
    for k in F.REG_FIELDS:
        tg[k] = ex[k].reshape(1, -1)
    cfg = {"w_bce": 1.0, "w_l2": 1.0}
    maps = []
    for graph_steps in (0, 3):
        m = lt.lt_map_create(32, 3, 1, lt.LT_ACT_TANH)
        lt.lt_map_set_params(m, torch.from_numpy(F.init_params(32, 3, 1, 9)).to(dev))
        s, loss = F.fit_epochs(m, rays, tg, 2, 4096, cfg, 21, lr=lambda k: 1e-3 * 0.9 ** k,
                               graph_steps=graph_steps)
        torch.cuda.synchronize()
        assert s == 16
        maps.append((m, loss.clone()))
    assert torch.equal(lt.lt_map_get_params(maps[0][0]), lt.lt_map_get_params(maps[1][0]))
    assert torch.equal(lt.lt_map_adam_state(maps[0][0]), lt.lt_map_adam_state(maps[1][0]))
    assert torch.equal(maps[0][1], maps[1][1])
