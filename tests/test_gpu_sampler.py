"""GPU parity of the training-data sampler: CIE wavelength sampling of the
device ray generator against the oracle's inverse CDF, and the device
Markov chains (lt_mcmc_run) against the oracle's chains on the same
counter-based uniforms.  Chains follow identical trajectories until a
proposal lands on a visibility boundary (where the FP32 tracer and the FP64
oracle may legitimately disagree); every divergence must be such a case."""
import numpy as np
import pytest

import oracle
import synth
from oracle import sampling as S

pytestmark = pytest.mark.gpu

HW, HH = synth.SENSOR_HALF_W, synth.SENSOR_HALF_H


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _uniforms(n, seed):
    ctr = np.arange(n, dtype=np.uint64)
    z = np.zeros(n, np.uint64)
    o0, o1, o2, o3 = synth.philox4x64_10((ctr, z, z, z), (seed, 0))
    m24 = np.uint64(0xFFFFFF)
    u4 = ((o0 >> np.uint64(16)) & m24).astype(np.float64) * 2.0 ** -24
    return u4


@pytest.mark.parametrize("lam_range", [(400.0, 700.0), (380.0, 780.0)])
def test_cie_wavelengths_match_oracle(dev, lam_range):
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    n = 200000
    g = lt.lt_rays_generate(h, n, 21, lam_range=lam_range, lambda_mode=lt.LT_LAMBDA_CIE)
    lam = g["lambda_nm"].cpu().numpy()
    torch.cuda.synchronize()
    ref = S.cie_inverse(_uniforms(n, 21), *lam_range)
    err = np.abs(lam.astype(np.float64) - ref)
    # FP32 rounding of the wavelength (half an ulp at 700 nm is 3e-5 nm)
    assert err.max() < 1e-4, err.max()
    # sensor points are those of the uniform mode, bit for bit
    twin = synth.philox_rays(L, n, 21, lam_range=lam_range)
    assert np.array_equal(g["x"].cpu().numpy(), twin["x"])
    print(f"[cie] {lam_range}: max |lambda - oracle| {err.max():.2e} nm", flush=True)


def _run_both(dev, L, path, n, steps, seed, lam_mode=0, split=None, p_large=0.1):
    import torch
    import paper_2605_04017_amd as lt
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    st = lt.lt_mcmc_init(lt.mcmc_state(n, dev), 0.05)
    calls = [(0, steps)] if split is None else [(0, split), (split, steps - split)]
    rays, exits, counts = [], [], None
    for first, k in calls:
        r, e, counts = lt.lt_mcmc_run(h, path, st, k, seed, first_step=first, p_large=p_large,
                                      lambda_mode=lam_mode, counts=counts)
        rays.append({f: v.cpu().numpy() for f, v in r.items()})
        exits.append({f: v.cpu().numpy() for f, v in e.items()})
    torch.cuda.synchronize()
    g_rays = {f: np.concatenate([r[f] for r in rays]) for f in rays[0]}
    g_exit = {f: np.concatenate([e[f] for e in exits]) for f in exits[0]}
    g_state = {k: v.cpu().numpy() for k, v in st.items()}
    vis = S.lens_visibility(L, path, HW, HH, lam_mode=lam_mode)
    ost = S.new_state(n, 0.05)
    props = []
    o_u, o_ok, o_counts = S.run_chains(vis, ost, seed, 0, steps, p_large=p_large, proposals=props)
    return g_rays, g_exit, g_state, counts.cpu().numpy(), o_u, o_ok, ost, o_counts, props


def _check_chains(L, path, n, steps, g_rays, g_exit, g_state, o_u, o_ok, ost, props, lam_mode=0):
    o_rays = [synth.rays_from_uniforms(L, o_u[t], HW, HH, lam=None if lam_mode == 0 else
                                       S.cie_inverse(o_u[t][4]).astype(np.float32)) for t in range(steps)]
    same_xy = np.stack([(g_rays["x"][t] == o_rays[t]["x"]) & (g_rays["y"][t] == o_rays[t]["y"]) &
                        (g_exit["mask"][t] == o_ok[t]) for t in range(steps)])
    ident = same_xy.all(0)
    # identical chains end in bit-identical states
    for k, ok in (("u", None), ("step", "d"), ("n_small", "m"), ("visible", "vis")):
        gv = g_state[k][:, ident] if k == "u" else g_state[k][ident]
        ov = ost["u"][:, ident] if k == "u" else ost[ok][ident]
        assert np.array_equal(gv.astype(np.float64), ov.astype(np.float64)), k
    # every divergence starts at a proposal on a visibility boundary
    bad = []
    for c in np.flatnonzero(~ident):
        t = int(np.argmin(same_xy[:, c]))
        p = props[t][:, c:c + 1]
        lam = None if lam_mode == 0 else S.cie_inverse(p[4]).astype(np.float32)
        r = synth.rays_from_uniforms(L, p, HW, HH, lam=lam)
        d = oracle.trace(L, r, path, diag=True)
        near = (d["edge_margin"][0] < 1e-4 or d["tir_margin"][0] < 1e-6 or d["graze_margin"][0] < 1e-9)
        if not near:
            bad.append((int(c), t, float(d["edge_margin"][0]), float(d["tir_margin"][0])))
    assert not bad, f"divergences away from a boundary: {bad[:5]}"
    # exit rays of the outputs: the tracer's parity on the identical chains
    both = (g_exit["mask"] == 1) & ident[None, :]
    tt, cc = np.nonzero(both)
    sel = np.arange(tt.size)[:: max(1, tt.size // 20000)]
    rays = {f: g_rays[f][tt[sel], cc[sel]] for f in synth.RAY_FIELDS}
    o = oracle.trace(L, rays, path)
    ok = o["mask"] == 1
    # the oracle traces the device's FP32 rays here, not its own FP64 ones,
    # so a boundary ray may flip; positions agree to the tracer's tolerance
    assert ok.mean() > 0.999
    pos = np.hypot(g_exit["x"][tt[sel], cc[sel]][ok] - o["x"][ok], g_exit["y"][tt[sel], cc[sel]][ok] - o["y"][ok])
    assert pos.max() < 1e-5
    return float(ident.mean())


@pytest.mark.parametrize("path,n,steps,split", [((1, 2, 10), 4096, 48, 20), ((0, 0, 0), 2048, 32, None)])
def test_mcmc_chains_match_oracle(dev, path, n, steps, split):
    L = synth.config_lens(2)
    g_rays, g_exit, g_state, g_counts, o_u, o_ok, ost, o_counts, props = _run_both(
        dev, L, path, n, steps, 33, split=split)
    frac = _check_chains(L, path, n, steps, g_rays, g_exit, g_state, o_u, o_ok, ost, props)
    assert frac > 0.98, frac
    # counts agree to the diverging chains
    assert np.abs(g_counts.astype(np.int64) - o_counts).max() <= 4 * (1 - frac) * n * steps + 4
    print(f"[mcmc] {path}: {frac:.4f} of {n} chains identical over {steps} steps; counts "
          f"{g_counts.tolist()} vs {o_counts.tolist()}", flush=True)


def test_mcmc_cie_chains_match_oracle(dev):
    L = synth.config_lens(2)
    path, n, steps = (1, 4, 10), 1024, 24
    g_rays, g_exit, g_state, _, o_u, o_ok, ost, _, props = _run_both(dev, L, path, n, steps, 44, lam_mode=1)
    frac = _check_chains(L, path, n, steps, g_rays, g_exit, g_state, o_u, o_ok, ost, props, lam_mode=1)
    assert frac > 0.97, frac


def test_mcmc_yield_and_normalisation(dev):
    """On a ghost with ~2 % valid uniform rays, the chains' outputs are
    valid after burn-in (a chain needs ~1/0.023 independent proposals to
    find its first valid state) at a rate far above rejection sampling, and
    the independent proposals' acceptance estimates the uniform valid
    fraction (the normalisation estimate of the adaptive chain)."""
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    path, n, steps = (1, 2, 10), 16384, 256
    st = lt.lt_mcmc_init(lt.mcmc_state(n, dev), 0.05)
    rays, ex, counts = lt.lt_mcmc_run(h, path, st, steps, 7)
    uni = lt.lt_rays_generate(h, 1 << 22, 8)
    f_uni = float(lt.lt_trace(h, path, uni)["mask"].float().mean())
    torch.cuda.synchronize()
    cnt = counts.cpu().numpy().astype(np.float64)
    p_hat = cnt[1] / cnt[0]
    assert abs(p_hat - f_uni) < 4 * np.sqrt(f_uni * (1 - f_uni) / cnt[0]) + 4 * np.sqrt(f_uni / (1 << 22))
    valid_after = float(ex["mask"][192:].float().mean())
    assert valid_after > 0.95
    small_acc = cnt[3] / cnt[2]
    print(f"[mcmc] yield: uniform valid fraction {f_uni:.4f}, estimate {p_hat:.4f}, small-step "
          f"acceptance {small_acc:.3f}, valid outputs after 192 steps {valid_after:.4f}", flush=True)


def test_mcmc_full_size_sampled(dev):
    """The benchmark configuration (1,048,576 chains on ghost (1, 2, 10)),
    64 steps from the initial state; 3,000 chains picked at random are
    followed by the oracle on their own counters."""
    import torch
    import paper_2605_04017_amd as lt
    L = synth.config_lens(2)
    h = lt.lt_lens_create(L.surfaces, L.glasses)
    path, n, steps, seed = (1, 2, 10), 1 << 20, 64, 7007
    st = lt.lt_mcmc_init(lt.mcmc_state(n, dev), 0.05)
    rays, ex, _ = lt.lt_mcmc_run(h, path, st, steps, seed)
    ids = np.sort(np.random.default_rng(1).choice(n, 3000, replace=False))
    idx = torch.from_numpy(ids).to(dev)
    g_x = rays["x"][:, idx].cpu().numpy()
    g_m = ex["mask"][:, idx].cpu().numpy()
    g_u = st["u"][:, idx].cpu().numpy()
    g_d = st["step"][idx].cpu().numpy()
    torch.cuda.synchronize()
    ost = S.new_state(ids.size, 0.05)
    o_u, o_ok, _ = S.run_chains(S.lens_visibility(L, path, HW, HH), ost, seed, 0, steps, chain_ids=ids)
    o_x = np.stack([synth.rays_from_uniforms(L, o_u[t], HW, HH)["x"] for t in range(steps)])
    ident = ((g_x == o_x) & (g_m == o_ok)).all(0)
    assert ident.mean() > 0.98, ident.mean()
    assert np.array_equal(g_u[:, ident], ost["u"][:, ident])
    assert np.array_equal(g_d[ident], ost["d"][ident])
    print(f"[mcmc] full size: {ident.mean():.4f} of 3,000 sampled chains identical", flush=True)
