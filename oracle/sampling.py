"""Training-data sampler of the data-collection step (Sec. 5.1): wavelength
importance sampling by the CIE XYZ colour-matching functions, and a Markov
chain over the primary sample space whose target is the binary visibility
of a path (Hachisuka and Jensen, "Robust adaptive photon tracing using
photon path visibility", ACM TOG 30(5), 2011).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

Colour matching functions: the multi-lobe analytic fit of Wyman, Sloan and
Shirley ("Simple analytic approximations to the CIE XYZ color matching
functions", JCGT 2(2), 2013): sums of split Gaussians
g(l; mu, s1, s2) = exp(-(l - mu)^2 / (2 s^2)), s = s1 left of mu, s2 right.
Wavelengths are drawn with density proportional to xbar + ybar + zbar on
[lambda_min, lambda_max] by inverting its closed-form CDF (erf) with
bisection in FP64.

Markov chain (one per lane on the device, vectorised here): the state is a
point u of [0, 1)^5 (sensor point x, y; target point radius and angle on
the rear disk; wavelength), mapped to a sensor-side ray by the ray recipe
of ``synth``.  Each step draws eight 24-bit uniforms from Philox4x64-10,
counter (step, chain, 1, 0), key (seed, 0):

* r_sel = bits 40..63 of word 0; c_0..c_4 = bits 16..39 of word 0, then
  bits 40..63 and 16..39 of words 1 and 2;
* a chain that holds no visible state, or one with r_sel < p_large, proposes
  the independent point u' = c (a "large step");
* otherwise u'_i = wrap(u_i + d * (2 c_i - 1)) (a "small step"), with
  wrap(v) = v - floor(v), mapped to 0 if it rounds to 1, in FP32;
* the proposal is accepted iff its path is valid (binary target, symmetric
  proposals: the Metropolis ratio is the visibility of u');
* after a small step the step size follows the Robbins-Monro rule of the
  adaptive chain, d <- d + (a - a*) / m (a = 1 if accepted, m = number of
  small steps so far, a* the target acceptance), clamped to [1e-5, 0.5];
  the update is FP32 with one rounding per operation, so both sides keep
  bit-identical step sizes;
* the step's output is the chain's state after the step (a repeat if the
  proposal was rejected), or the rejected proposal, marked invalid, while
  the chain has not yet found a visible state.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, Tuple

import numpy as np

# (weight, mu, sigma_left, sigma_right) per lobe
_XBAR = ((1.056, 599.8, 37.9, 31.0), (0.362, 442.0, 16.0, 26.7), (-0.065, 501.1, 20.4, 26.2))
_YBAR = ((0.821, 568.8, 46.9, 40.5), (0.286, 530.9, 16.3, 31.1))
_ZBAR = ((1.217, 437.0, 11.8, 36.0), (0.681, 459.0, 26.0, 13.8))
_LOBES = _XBAR + _YBAR + _ZBAR

STEP_MIN, STEP_MAX = 1e-5, 0.5


def _lobe(l, mu, s1, s2):
    s = np.where(np.asarray(l) < mu, s1, s2)
    return np.exp(-0.5 * ((np.asarray(l, np.float64) - mu) / s) ** 2)


def cmf(l) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(xbar, ybar, zbar) of the analytic fit at wavelengths l (nm)."""
    return tuple(sum(w * _lobe(l, mu, s1, s2) for w, mu, s1, s2 in lobes)
                 for lobes in (_XBAR, _YBAR, _ZBAR))


def cie_density(l) -> np.ndarray:
    """xbar + ybar + zbar (unnormalised sampling density)."""
    return sum(w * _lobe(l, mu, s1, s2) for w, mu, s1, s2 in _LOBES)


def _lobe_integral(l, mu: float, s1: float, s2: float):
    """Integral of one split Gaussian from -inf to l (scalar or array)."""
    from scipy.special import erf, erfc
    c = math.sqrt(math.pi / 2.0)
    l = np.asarray(l, np.float64)
    left = s1 * c * erfc((mu - l) / (s1 * math.sqrt(2.0)))
    right = s1 * c + s2 * c * erf((l - mu) / (s2 * math.sqrt(2.0)))
    return np.where(l < mu, left, right)


def cie_cdf(l):
    """Closed-form integral of cie_density from -inf to l."""
    v = sum(w * _lobe_integral(l, mu, s1, s2) for w, mu, s1, s2 in _LOBES)
    return float(v) if np.ndim(v) == 0 else v


def cie_inverse(u, lam_min: float = 400.0, lam_max: float = 700.0) -> np.ndarray:
    """Wavelengths with density proportional to cie_density on
    [lam_min, lam_max]: the root of cdf(l) = cdf(lo) + u (cdf(hi) - cdf(lo)),
    by 64 bisection steps in FP64."""
    u = np.atleast_1d(np.asarray(u, np.float64))
    f0, f1 = cie_cdf(lam_min), cie_cdf(lam_max)
    tgt = f0 + u * (f1 - f0)
    lo = np.full(u.shape, float(lam_min))
    hi = np.full(u.shape, float(lam_max))
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        below = cie_cdf(mid) < tgt
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


# ------------------------------------------------------------ the chain ----

def step_uniforms(seed: int, step: int, chains: np.ndarray):
    """(r_sel, c[5, n]) of one step for the given chain indices."""
    import synth
    n = chains.shape[0]
    ctr = (np.full(n, step, np.uint64), chains.astype(np.uint64), np.ones(n, np.uint64),
           np.zeros(n, np.uint64))
    w0, w1, w2, _ = synth.philox4x64_10(ctr, (seed, 0))
    m24 = np.uint64(0xFFFFFF)

    def hi(w):
        return ((w >> np.uint64(40)) & m24).astype(np.float32) * np.float32(2.0 ** -24)

    def lo(w):
        return ((w >> np.uint64(16)) & m24).astype(np.float32) * np.float32(2.0 ** -24)
    return hi(w0), np.stack([lo(w0), hi(w1), lo(w1), hi(w2), lo(w2)])


def wrap(v: np.ndarray) -> np.ndarray:
    """v - floor(v) in FP32, with a result that rounds to 1 mapped to 0."""
    v = np.asarray(v, np.float32)
    w = (v - np.floor(v)).astype(np.float32)
    return np.where(w >= np.float32(1.0), np.float32(0.0), w).astype(np.float32)


def run_chains(visible: Callable[[np.ndarray], np.ndarray], state: Dict[str, np.ndarray],
               seed: int, first_step: int, n_steps: int, p_large: float = 0.1,
               target: float = 0.234, proposals: list | None = None,
               chain_ids: np.ndarray | None = None):
    """Advance every chain by n_steps.  ``visible(u)`` maps a (5, n) FP32
    array of primary-sample points to their boolean visibility.  ``state``
    (modified in place): u (5, n) float32, d (n,) float32, m (n,) int32,
    vis (n,) bool.  Returns per-step outputs: u (n_steps, 5, n), valid
    (n_steps, n), and the counts [large proposals, large accepted, small
    proposals, small accepted].  If ``proposals`` is a list, each step's
    proposals (5, n) are appended to it.  ``chain_ids`` gives the chains'
    indices in the counter (default 0..n-1), so any subset of a large run
    can be followed on its own."""
    f32 = np.float32
    u, d, m, vis = state["u"], state["d"], state["m"], state["vis"]
    n = u.shape[1]
    chains = np.arange(n) if chain_ids is None else np.asarray(chain_ids, np.int64)
    out_u = np.empty((n_steps, 5, n), np.float32)
    out_ok = np.empty((n_steps, n), bool)
    counts = np.zeros(4, np.int64)
    pl, tg = f32(p_large), f32(target)
    for t in range(n_steps):
        r_sel, c = step_uniforms(seed, first_step + t, chains)
        large = ~vis | (r_sel < pl)
        small_prop = wrap(u + d[None, :] * (f32(2.0) * c - f32(1.0)))
        prop = np.where(large[None, :], c, small_prop).astype(f32)
        if proposals is not None:
            proposals.append(prop.copy())
        acc = visible(prop)
        counts += [large.sum(), (large & acc).sum(), (~large).sum(), (~large & acc).sum()]
        sm = ~large
        m[sm] += 1
        a = np.where(acc, f32(1.0), f32(0.0)).astype(f32)
        with np.errstate(divide="ignore", invalid="ignore"):
            upd = (d + (a - tg) / m.astype(f32)).astype(f32)
        d[:] = np.where(sm, np.clip(upd, f32(STEP_MIN), f32(STEP_MAX)), d).astype(f32)
        u[:, acc] = prop[:, acc]
        vis |= acc
        out_u[t] = np.where(vis[None, :], u, prop)
        out_ok[t] = vis
    return out_u, out_ok, counts


def new_state(n: int, d0: float = 0.05) -> Dict[str, np.ndarray]:
    return {"u": np.zeros((5, n), np.float32), "d": np.full(n, d0, np.float32),
            "m": np.zeros(n, np.int32), "vis": np.zeros(n, bool)}


def lens_visibility(lens, path, half_w: float, half_h: float, lam_range=(400.0, 700.0),
                    lam_mode: int = 0):
    """visible(u) for a lens path: the sensor-side ray of each point (the
    recipe of ``synth.rays_from_uniforms``) traced by the FP64 oracle."""
    import oracle
    import synth

    def vis(u):
        lam = None
        if lam_mode == 1:
            lam = cie_inverse(u[4], *lam_range).astype(np.float32)
        rays = synth.rays_from_uniforms(lens, u, half_w, half_h, lam_range, lam)
        return oracle.trace(lens, rays, tuple(path))["mask"] == 1
    return vis
