"""Brute-force pin of the FP64 oracle on tiny lenses.

An independent 40-digit tracer written with mpmath from a different
formulation: the sphere in centre form |q - C| = |R|, refraction as a
rotation in the plane of incidence by the Snell angle (sin t = eta sin i),
Fresnel factors from the angle-form (sine/tangent) laws.  Agreement is
required to 1e-11 mm / 1e-12 on direction components / 1e-13 on throughput
for rays farther than 1e-9 mm from any aperture edge.
"""
import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

import oracle
import synth
from synth import Glass, Lens, Surface

mp.mp.dps = 40


def _index(glass, lam_nm):
    lam = mp.mpf(float(lam_nm)) / 1000
    if glass.kind == 0:
        return mp.mpf(1)
    if glass.kind == 1:
        a, b, c = (mp.mpf(v) for v in glass.coef[:3])
        return a + b / lam ** 2 + c / lam ** 4
    s = mp.mpf(1)
    for bb, cc in zip(glass.coef[:3], glass.coef[3:]):
        s += mp.mpf(bb) * lam ** 2 / (lam ** 2 - mp.mpf(cc))
    return mp.sqrt(s)


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _unit(a):
    n = mp.sqrt(_dot(a, a))
    return [a[0] / n, a[1] / n, a[2] / n]


def bf_trace(lens, path, x, y, dx, dy, dz, lam):
    """Independent tracer; returns (valid, p, d, I, min_edge_margin)."""
    surfs = lens.surfaces
    zv = [mp.mpf(0)]
    for s in surfs[:-1]:
        zv.append(zv[-1] + mp.mpf(s.thickness))
    zs = zv[-1] + mp.mpf(surfs[-1].thickness)
    nmed = [mp.mpf(1)] + [_index(lens.glasses[s.glass_after], lam) for s in surfs]
    # interaction list: (surface, kind) with kind T/R/S and the incoming side
    refr = [k for k, s in enumerate(surfs) if not s.is_stop]
    seq = []
    kind, j, i = path
    if kind == 0:
        seq = [(k, "S" if surfs[k].is_stop else "T", -1) for k in range(len(surfs) - 1, -1, -1)]
    else:
        sj, si = refr[j - 1], refr[i - 1]
        seq += [(k, "S" if surfs[k].is_stop else "T", -1) for k in range(len(surfs) - 1, sj, -1)]
        seq += [(sj, "R", -1)]
        seq += [(k, "S" if surfs[k].is_stop else "T", +1) for k in range(sj + 1, si)]
        seq += [(si, "R", +1)]
        seq += [(k, "S" if surfs[k].is_stop else "T", -1) for k in range(si - 1, -1, -1)]
    p = [mp.mpf(float(x)), mp.mpf(float(y)), zs]
    d = _unit([mp.mpf(float(dx)), mp.mpf(float(dy)), mp.mpf(float(dz))])
    I = mp.mpf(1)
    margin = mp.inf
    for (k, ty, side) in seq:
        s = surfs[k]
        if s.radius == 0.0:
            if d[2] == 0:
                return False, None, None, 0, margin
            t = (zv[k] - p[2]) / d[2]
            if t <= 0:
                return False, None, None, 0, margin
            q = [p[0] + t * d[0], p[1] + t * d[1], zv[k]]
            nrm = [mp.mpf(0), mp.mpf(0), mp.mpf(-1)]
        else:
            R = mp.mpf(s.radius)
            Cc = [mp.mpf(0), mp.mpf(0), zv[k] + R]
            w = [p[0] - Cc[0], p[1] - Cc[1], p[2] - Cc[2]]
            b = _dot(d, w)
            cc = _dot(w, w) - R * R
            disc = b * b - cc
            if disc < 0:
                return False, None, None, 0, margin
            best = None
            for t in (-b - mp.sqrt(disc), -b + mp.sqrt(disc)):
                q = [p[0] + t * d[0], p[1] + t * d[1], p[2] + t * d[2]]
                # vertex hemisphere: the hit lies on the vertex side of the centre
                if t > 0 and (q[2] - Cc[2]) / R < 0 and (best is None or t < best[0]):
                    best = (t, q)
            if best is None:
                return False, None, None, 0, margin
            t, q = best
            nrm = _unit([q[0] - Cc[0], q[1] - Cc[1], q[2] - Cc[2]])
        h = mp.sqrt(q[0] ** 2 + q[1] ** 2)
        margin = min(margin, abs(h - mp.mpf(s.semi_diameter)))
        if h > mp.mpf(s.semi_diameter):
            return False, None, None, 0, margin
        p = q
        if ty == "S":
            continue
        if _dot(nrm, d) > 0:
            nrm = [-nrm[0], -nrm[1], -nrm[2]]
        ci = -_dot(nrm, d)
        ti = mp.acos(min(mp.mpf(1), ci))
        n1, n2 = (nmed[k + 1], nmed[k]) if side < 0 else (nmed[k], nmed[k + 1])
        tang = [d[0] + ci * nrm[0], d[1] + ci * nrm[1], d[2] + ci * nrm[2]]
        tl = mp.sqrt(_dot(tang, tang))
        u = [tang[0] / tl, tang[1] / tl, tang[2] / tl] if tl > 0 else [0, 0, 0]
        st = n1 / n2 * mp.sin(ti)
        if ty == "T":
            if st > 1:
                return False, None, None, 0, margin
            tt = mp.asin(st)
            d = [-mp.cos(tt) * nrm[m] + mp.sin(tt) * u[m] for m in range(3)]
            if ti == 0:
                Tf = 4 * n1 * n2 / (n1 + n2) ** 2
            else:
                ts = 2 * mp.sin(tt) * mp.cos(ti) / mp.sin(ti + tt)
                tp = 2 * mp.sin(tt) * mp.cos(ti) / (mp.sin(ti + tt) * mp.cos(ti - tt))
                Tf = n2 * mp.cos(tt) / (n1 * mp.cos(ti)) * (ts ** 2 + tp ** 2) / 2
            I *= Tf
        else:
            d = [mp.cos(ti) * nrm[m] + mp.sin(ti) * u[m] for m in range(3)]
            if st > 1:
                Rf = mp.mpf(1)
            elif ti == 0:
                Rf = ((n1 - n2) / (n1 + n2)) ** 2
            else:
                tt = mp.asin(st)
                rs = -mp.sin(ti - tt) / mp.sin(ti + tt)
                rp = mp.tan(ti - tt) / mp.tan(ti + tt)
                Rf = (rs ** 2 + rp ** 2) / 2
            I *= Rf
    if d[2] >= 0:
        return False, None, None, 0, margin
    t = (0 - p[2]) / d[2]
    q = [p[0] + t * d[0], p[1] + t * d[1], mp.mpf(0)]
    return True, q, d, I, margin


def _tiny_lenses():
    rng = np.random.default_rng(123)
    lenses = []
    air = Glass(0, [0.0] * 6)
    for k in range(3):
        g = Glass(1, [rng.uniform(1.5, 1.75), rng.uniform(0.003, 0.015), 0, 0, 0, 0])
        r1 = rng.uniform(25, 60) * (1 if k != 1 else -1)
        lenses.append(Lens([Surface(r1, 30.0, 12.0, 1, 0)], [air, g]))
        r2 = -rng.uniform(30, 80)
        lenses.append(Lens([Surface(abs(r1), rng.uniform(4, 8), 12.0, 1, 0),
                            Surface(r2, 40.0, 12.0, 0, 0)], [air, g]))
    gs = Glass(2, [1.03961212, 0.231792344, 1.01046945, 0.00600069867, 0.0200179144, 103.560653])
    lenses.append(Lens([Surface(40.0, 6.0, 14.0, 1, 0), Surface(0.0, 5.0, 6.0, 0, 1),
                        Surface(-35.0, 45.0, 14.0, 0, 0)], [air, gs]))
    lenses.append(synth.config_lens(1))
    return lenses


@pytest.mark.parametrize("li", range(8))
def test_bruteforce_agreement(li):
    lens = _tiny_lenses()[li]
    rays = synth.make_rays(lens, 60, 900 + li)
    nr = lens.n_refracting
    paths = [(0, 0, 0)] + ([(1, 1, nr)] if nr >= 2 else [])
    agree = 0
    for path in paths:
        o = oracle.trace(lens, rays, path=path)
        for r in range(60):
            ok, p, d, I, margin = bf_trace(lens, path, rays["x"][r], rays["y"][r], rays["dx"][r],
                                           rays["dy"][r], rays["dz"][r], rays["lambda_nm"][r])
            if margin < 1e-9:
                continue
            assert bool(o["mask"][r]) == ok, (li, path, r)
            if ok:
                assert abs(float(p[0]) - o["x"][r]) < 1e-11
                assert abs(float(p[1]) - o["y"][r]) < 1e-11
                assert abs(float(d[0]) - o["dx"][r]) < 1e-12
                assert abs(float(d[1]) - o["dy"][r]) < 1e-12
                assert abs(float(d[2]) - o["dz"][r]) < 1e-12
                assert abs(float(I) - o["throughput"][r]) < 1e-13
                agree += 1
    assert agree >= 10
