"""Pins of the oracle's training-data sampler (Sec. 5.1 data collection):
the CIE colour-matching fit against the CIE 1931 standard observer, its
closed-form CDF against numerical quadrature, the wavelength inverse, and
the visibility-target Markov chain against facts that hold for any correct
sampler (uniform stationary distribution on the visible set, the large-step
acceptance estimating the visible volume, step-size adaptation reaching its
target acceptance, independent proposals reducing to rejection sampling)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import sampling as S

# CIE 1931 2-degree standard observer (xbar, ybar, zbar) at a few wavelengths
CIE1931 = {400: (0.01431, 0.00040, 0.06785), 450: (0.33620, 0.03800, 1.77211),
           500: (0.00490, 0.32300, 0.27200), 550: (0.43345, 0.99500, 0.00875),
           555: (0.51205, 1.00000, 0.00575), 600: (1.06220, 0.63100, 0.00080),
           650: (0.28350, 0.10700, 0.00000), 700: (0.01136, 0.00410, 0.00000)}


def test_cmf_fit_matches_cie_1931():
    """The analytic fit stays within 0.012 of the standard table (its
    published accuracy is of that order; a swapped width or a wrong weight
    moves some value by several times more)."""
    for lam, ref in CIE1931.items():
        got = [float(v) for v in S.cmf(lam)]
        assert max(abs(a - b) for a, b in zip(got, ref)) < 0.012, (lam, got, ref)
    # ybar peaks near 555 nm at about 1
    grid = np.linspace(380, 780, 4001)
    yb = S.cmf(grid)[1]
    assert abs(grid[np.argmax(yb)] - 556) < 6 and abs(yb.max() - 1.0) < 0.01


def test_cdf_closed_form_matches_quadrature():
    """Split the quadrature at every lobe centre (where the widths switch)."""
    mus = sorted({lobe[1] for lobe in S._LOBES})
    for lam in (380.0, 437.0, 480.0, 501.1, 568.8, 620.0, 780.0):
        pts = [0.0] + [m for m in mus if m < lam] + [lam]
        num = sum(integrate.quad(S.cie_density, a, b, epsabs=1e-13, epsrel=1e-13, limit=200)[0]
                  for a, b in zip(pts[:-1], pts[1:]))
        num += integrate.quad(S.cie_density, -np.inf, 0.0)[0]
        assert math.isclose(S.cie_cdf(lam), num, rel_tol=1e-11, abs_tol=1e-11), lam
    # density is positive across the sampled range
    g = np.linspace(380, 780, 2001)
    assert np.all(S.cie_density(g) > 0)


def test_inverse_is_the_cdf_inverse_and_samples_the_density():
    lo, hi = 400.0, 700.0
    u = (np.arange(20000) + 0.5) / 20000
    lam = S.cie_inverse(u, lo, hi)
    assert np.all(np.diff(lam) > 0) and lam[0] > lo and lam[-1] < hi
    f0, f1 = S.cie_cdf(lo), S.cie_cdf(hi)
    back = np.array([(S.cie_cdf(v) - f0) / (f1 - f0) for v in lam[::97]])
    assert np.abs(back - u[::97]).max() < 1e-12
    # stratified u: each 10 nm bin holds its share of the density
    edges = np.arange(lo, hi + 1e-9, 10.0)
    share = np.array([integrate.quad(S.cie_density, a, b)[0] for a, b in zip(edges[:-1], edges[1:])])
    share /= share.sum()
    frac = np.histogram(lam, edges)[0] / lam.size
    assert np.abs(frac - share).max() < 2e-4
    assert S.cie_inverse([0.0], lo, hi)[0] == pytest.approx(lo, abs=1e-9)
    assert S.cie_inverse([1.0], lo, hi)[0] == pytest.approx(hi, abs=1e-9)


def test_wrap():
    v = np.array([0.75, 1.25, -0.25, -1e-9, 1.0, 0.0, 1.5 - 2 ** -23], np.float32)
    w = S.wrap(v)
    assert w.dtype == np.float32
    assert w.tolist() == [0.75, 0.25, 0.75, 0.0, 0.0, 0.0, 0.5 - 2 ** -23]
    assert np.all((w >= 0) & (w < 1))


def _annulus(u):
    r2 = (u[0] - 0.5) ** 2 + (u[1] - 0.5) ** 2
    return (r2 >= 0.04) & (r2 <= 0.16)


def test_independent_proposals_reduce_to_rejection_sampling():
    """p_large = 1: every step proposes a fresh uniform point; the chain's
    output is the latest visible proposal, which a plain loop over the same
    uniforms reproduces."""
    n, T = 200, 30
    st = S.new_state(n)
    out_u, ok, counts = S.run_chains(_annulus, st, seed=5, first_step=0, n_steps=T, p_large=1.0)
    assert counts[2] == 0 and counts[0] == n * T
    for c in (0, 7, 199):
        cur = None
        for t in range(T):
            _, cu = S.step_uniforms(5, t, np.array([c]))
            cand = cu[:, 0]
            if _annulus(cand[:, None])[0]:
                cur = cand
            if cur is None:
                assert not ok[t, c]
                assert np.array_equal(out_u[t, :, c], cand)
            else:
                assert ok[t, c] and np.array_equal(out_u[t, :, c], cur)


def test_chain_samples_the_visible_set_uniformly():
    """Binary target: after burn-in the states are uniform on the visible
    annulus, r^2 uniform on [0.04, 0.16], angle uniform, free coordinates
    uniform; the large-step acceptance estimates the annulus area
    pi (0.16 - 0.04) (the normalisation estimate of the adaptive chain)."""
    n, T = 4000, 120
    st = S.new_state(n)
    out_u, ok, counts = S.run_chains(_annulus, st, seed=11, first_step=0, n_steps=T, p_large=0.1)
    tail = out_u[40:][:, :, ok[40:].all(0)]
    u = tail.transpose(1, 0, 2).reshape(5, -1)
    r2 = (u[0] - 0.5) ** 2 + (u[1] - 0.5) ** 2
    assert r2.min() >= 0.04 - 1e-7 and r2.max() <= 0.16 + 1e-7
    # states are correlated along a chain: test one sample per chain per 20 steps
    thin = tail[::20].transpose(1, 0, 2).reshape(5, -1)
    r2t = (thin[0] - 0.5) ** 2 + (thin[1] - 0.5) ** 2
    assert stats.kstest((r2t - 0.04) / 0.12, "uniform").pvalue > 1e-3
    ang = (np.arctan2(thin[1] - 0.5, thin[0] - 0.5) + np.pi) / (2 * np.pi)
    assert stats.kstest(ang, "uniform").pvalue > 1e-3
    for k in (2, 3, 4):
        assert stats.kstest(thin[k], "uniform").pvalue > 1e-3
    area = math.pi * 0.12
    p_hat = counts[1] / counts[0]
    # large steps of still-empty chains are part of the same uniform stream
    assert abs(p_hat - area) < 4 * math.sqrt(area * (1 - area) / counts[0])


def _thin_annulus(u):
    r2 = (u[0] - 0.5) ** 2 + (u[1] - 0.5) ** 2
    return (r2 >= 0.0225) & (r2 <= 0.04)


def test_step_size_adapts_to_target_acceptance():
    """On a visible set of volume 0.055 (below the target acceptance, so the
    target is reachable), the Robbins-Monro rule brings the small-step
    acceptance to 0.234.  (On a set larger than the target no step size can
    get there: a step size of 0.5 already proposes uniformly.)"""
    n, T = 2000, 300
    st = S.new_state(n, d0=0.5)
    S.run_chains(_thin_annulus, st, seed=12, first_step=0, n_steps=T, p_large=0.05)
    _, _, c2 = S.run_chains(_thin_annulus, st, seed=12, first_step=T, n_steps=100, p_large=0.05)
    acc = c2[3] / c2[2]
    assert abs(acc - 0.234) < 0.02, acc
    assert np.all((st["d"] >= S.STEP_MIN) & (st["d"] <= S.STEP_MAX))
    # on the larger annulus the step size runs to its cap
    st = S.new_state(500, d0=0.1)
    S.run_chains(_annulus, st, seed=13, first_step=0, n_steps=200, p_large=0.05)
    assert np.median(st["d"]) > 0.45


def test_chain_runs_resume_exactly():
    """Splitting a run into two calls (first_step offset) gives the same
    states and step sizes as one call: the counter-based uniforms depend
    only on (seed, step, chain)."""
    n = 300
    a = S.new_state(n)
    ua, oka, _ = S.run_chains(_annulus, a, seed=3, first_step=0, n_steps=50)
    b = S.new_state(n)
    ub1, okb1, _ = S.run_chains(_annulus, b, seed=3, first_step=0, n_steps=20)
    ub2, okb2, _ = S.run_chains(_annulus, b, seed=3, first_step=20, n_steps=30)
    assert np.array_equal(ua, np.concatenate([ub1, ub2]))
    for k in a:
        assert np.array_equal(a[k], b[k])
