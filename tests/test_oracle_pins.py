"""Pins for the FP64 oracle tracer against closed forms and invariants.

Each test checks the oracle against something other than itself: textbook
closed forms of refraction and Fresnel reflection, first-order (ABCD) optics,
the symmetry property of Sec. 4.1, reversibility of sequential tracing and
published glass data.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from synth import Glass, Lens, Surface

AIR = Glass(0, [0.0] * 6)


def cauchy(a, b, c=0.0):
    return Glass(1, [a, b, c, 0.0, 0.0, 0.0])


def plate(n=1.5, t=5.0, back=20.0, sd=30.0, stop_sd=None):
    """Flat glass plate: surface 1 at z=0, surface 2 at z=t, sensor at z=t+back."""
    surfs = [Surface(0.0, t, sd, 1, 0), Surface(0.0, back, sd, 0, 0)]
    if stop_sd is not None:
        surfs = [Surface(0.0, t, sd, 1, 0), Surface(0.0, back / 2, sd, 0, 0),
                 Surface(0.0, back / 2, stop_sd, 0, 1)]
    return Lens(surfs, [AIR, cauchy(n, 0.0)])


def one_ray(x, y, dx, dy, dz, lam=550.0):
    f = np.float32
    return {"x": np.array([x], f), "y": np.array([y], f), "dx": np.array([dx], f),
            "dy": np.array([dy], f), "dz": np.array([dz], f), "lambda_nm": np.array([lam], f)}


def fresnel_sine_law(n1, n2, ti):
    """R and T from Fresnel's sine/tangent laws (angle form), for a pin."""
    st = n1 / n2 * math.sin(ti)
    tt = math.asin(st)
    if ti == 0.0:
        r = (n1 - n2) / (n1 + n2)
        return r * r, 1 - r * r, tt
    rs = -math.sin(ti - tt) / math.sin(ti + tt)
    rp = math.tan(ti - tt) / math.tan(ti + tt)
    ts = 2 * math.sin(tt) * math.cos(ti) / math.sin(ti + tt)
    tp = 2 * math.sin(tt) * math.cos(ti) / (math.sin(ti + tt) * math.cos(ti - tt))
    fac = n2 * math.cos(tt) / (n1 * math.cos(ti))
    return 0.5 * (rs * rs + rp * rp), 0.5 * fac * (ts * ts + tp * tp), tt


# ---------------------------------------------------------------- Fresnel --

@pytest.mark.parametrize("n", [1.5, 1.72, 1.9])
def test_normal_incidence_plate(n):
    """On-axis through a plate: T = (4n/(n+1)^2)^2, direction unchanged."""
    L = plate(n=n)
    o = oracle.trace(L, one_ray(0, 0, 0, 0, -1))
    assert o["mask"][0] == 1
    t1 = 4 * n / (n + 1) ** 2
    assert abs(o["throughput"][0] - t1 * t1) < 1e-15
    assert o["x"][0] == 0 and o["y"][0] == 0 and o["dz"][0] == -1.0


@pytest.mark.parametrize("theta_deg", [0.0, 10.0, 35.0, 56.0, 70.0, 85.0])
@pytest.mark.parametrize("n", [1.5, 1.8])
def test_single_interface_R_T(theta_deg, n):
    """One air/glass interface hit from the air side at angle theta.

    T from the oracle's transmission step, R from its reflection step; both
    against Fresnel's angle-form equations, and R + T = 1.
    """
    L = plate(n=n, t=5.0, back=20.0, sd=1e6)
    zs = L.sensor_z
    th = math.radians(theta_deg)
    d = (math.sin(th), 0.0, -math.cos(th))
    o = (0.0, 0.0, zs)
    okT, _, dT, T, _ = oracle.trace_sequence(L, [(1, 0, -1)], 550.0, o, d, 2.0, -1)
    okR, _, dR, R, _ = oracle.trace_sequence(L, [(1, 1, -1)], 550.0, o, d, zs, +1)
    assert okT and okR
    R0, T0, tt = fresnel_sine_law(1.0, n, th)
    assert abs(T - T0) < 1e-14
    assert abs(R - R0) < 1e-14
    assert abs(R + T - 1.0) < 1e-14
    # Snell's law in angle form and mirror reflection
    assert abs(math.asin(dT[0]) - tt) < 1e-13
    assert abs(dR[0] - d[0]) < 1e-15 and abs(dR[2] + d[2]) < 1e-15


def test_brewster_angle():
    n = 1.6
    tb = math.atan(n)
    L = plate(n=n, sd=1e6)
    d = (math.sin(tb), 0.0, -math.cos(tb))
    ok, _, _, R, _ = oracle.trace_sequence(L, [(1, 1, -1)], 550.0, (0, 0, L.sensor_z), d,
                                           L.sensor_z, +1)
    tt = math.pi / 2 - tb
    rs = -math.sin(tb - tt) / math.sin(tb + tt)
    assert ok and abs(R - 0.5 * rs * rs) < 1e-14


def test_critical_angle_tir():
    """Glass -> air: below the critical angle transmits, above it dies (T step)
    and reflects everything (R step)."""
    n = 1.7
    tc = math.asin(1.0 / n)
    # medium after surface 2 is glass: sensor sits inside the glass
    L = Lens([Surface(0.0, 5.0, 1e6, 0, 0), Surface(0.0, 10.0, 1e6, 1, 0)], [AIR, cauchy(n, 0)])
    zs = L.sensor_z
    for th, expect in [(tc - 1e-6, True), (tc + 1e-6, False)]:
        d = (math.sin(th), 0.0, -math.cos(th))
        ok, _, _, _, dg = oracle.trace_sequence(L, [(1, 0, -1)], 550.0, (0, 0, zs), d, 0.0, -1)
        assert ok == expect
        if not expect:
            assert dg["fail_kind"] == 4
    d = (math.sin(tc + 0.1), 0.0, -math.cos(tc + 0.1))
    ok, _, _, R, _ = oracle.trace_sequence(L, [(1, 1, -1)], 550.0, (0, 0, zs), d, zs, +1)
    assert ok and R == 1.0


# ------------------------------------------------------------- geometry ----

@pytest.mark.parametrize("theta_deg", [5.0, 25.0, 50.0])
def test_plate_lateral_shift(theta_deg):
    n, t, back = 1.55, 6.0, 20.0
    L = plate(n=n, t=t, back=back, sd=1e6)
    th = math.radians(theta_deg)
    tt = math.asin(math.sin(th) / n)
    d = (math.sin(th) * math.cos(0.3), math.sin(th) * math.sin(0.3), -math.cos(th))
    ok, p, dout, I, _ = oracle.trace_sequence(L, oracle.build_sequence(L, 0), 550.0,
                                              (1.0, -2.0, t + back), d, 0.0, -1)
    assert ok
    assert np.allclose(dout, np.array(d) / np.linalg.norm(d), atol=1e-15)
    r = back * math.tan(th) + t * math.tan(tt)
    assert abs(p[0] - (1.0 + r * math.cos(0.3))) < 1e-12
    assert abs(p[1] - (-2.0 + r * math.sin(0.3))) < 1e-12
    # closed-form lateral displacement relative to the undeviated line
    shift = t * math.sin(th - tt) / math.cos(tt)
    undev = (t + back) * math.tan(th)
    assert abs((undev - r) * math.cos(th) - shift) < 1e-12
    R0, T0, _ = fresnel_sine_law(1.0, n, th)
    assert abs(I - T0 * T0) < 1e-14


@pytest.mark.parametrize("theta_deg", [0.0, 12.0, 30.0])
def test_plate_ghost_closed_form(theta_deg):
    """Ghost (1,2) in a plate: T, R, R, T; direction unchanged; three crossings."""
    n, t, back = 1.62, 4.0, 15.0
    L = plate(n=n, t=t, back=back, sd=1e6)
    th = math.radians(theta_deg)
    tt = math.asin(math.sin(th) / n)
    rays = one_ray(0.0, 0.0, math.sin(th), 0.0, -math.cos(th))
    th32 = math.acos(-float(rays["dz"][0]) / math.hypot(float(rays["dx"][0]), float(rays["dz"][0])))
    tt32 = math.asin(math.sin(th32) / n)
    o = oracle.trace(L, rays, path=(1, 1, 2))
    assert o["mask"][0] == 1
    R0, T0, _ = fresnel_sine_law(1.0, n, th32)
    assert abs(o["throughput"][0] - T0 * T0 * R0 * R0) < 1e-15
    x = back * math.tan(th32) + 3 * t * math.tan(tt32)
    assert abs(o["x"][0] - x) < 1e-12
    assert abs(o["dx"][0] - math.sin(th32)) < 1e-15


def test_ray_through_centre_undeviated():
    """A ray aimed at the centre of curvature meets the sphere normally."""
    n, R = 1.6, 40.0
    L = Lens([Surface(R, 70.0, 30.0, 1, 0)], [AIR, cauchy(n, 0)])
    zs = L.sensor_z
    rng = np.random.default_rng(0)
    for _ in range(20):
        x0, y0 = rng.uniform(-10, 10, 2)
        d = np.array([0.0 - x0, 0.0 - y0, R - zs])
        d /= np.linalg.norm(d)
        ok, p, dout, I, _ = oracle.trace_sequence(L, [(0, 0, -1)], 550.0, (x0, y0, zs), d, 0.0, -1)
        assert ok
        assert np.allclose(dout, d, atol=1e-14)
        assert abs(I - 4 * n / (n + 1) ** 2) < 1e-14


def test_stop_clips_closed_disk():
    L = plate(n=1.5, t=3.0, back=20.0, sd=30.0, stop_sd=2.0)
    zs = L.sensor_z
    # straight down the axis direction: h at the stop equals the start radius
    for x, expect in [(1.999, 1), (2.0, 1), (2.001, 0)]:
        o = oracle.trace(L, one_ray(x, 0, 0, 0, -1), diag=True)
        assert o["mask"][0] == expect, x
    o = oracle.trace(L, one_ray(2.5, 0, 0, 0, -1), diag=True)
    assert o["fail_kind"][0] == 3


# ------------------------------------------------------ whole-lens pins ---

def _lens_indices(L, lam):
    ns = [1.0]
    for s in L.surfaces:
        ns.append(oracle.glass_index(L, s.glass_after, lam))
    return ns


@pytest.mark.parametrize("config", [1, 2])
def test_on_axis_ray(config):
    """On-axis ray stays on axis; throughput is the product of normal-incidence T."""
    L = synth.config_lens(config)
    for lam in (450.0, 550.0, 650.0):
        o = oracle.trace(L, one_ray(0, 0, 0, 0, -1, lam))
        lam32 = float(np.float32(lam))
        ns = _lens_indices(L, lam32)
        Tprod = 1.0
        for k in range(len(L.surfaces)):
            a, b = ns[k], ns[k + 1]
            Tprod *= 4 * a * b / (a + b) ** 2
        assert o["mask"][0] == 1
        assert abs(o["x"][0]) < 1e-15 and abs(o["y"][0]) < 1e-15
        assert abs(o["dz"][0] + 1) < 1e-15
        assert abs(o["throughput"][0] - Tprod) < 1e-14


def _abcd(L, lam):
    """First-order system matrix (reduced angles) from the front vertex to the
    last vertex, written independently of the oracle."""
    ns = _lens_indices(L, lam)
    M = np.eye(2)
    zs = L.vertex_z
    for k, s in enumerate(L.surfaces):
        c = 0.0 if s.radius == 0 else 1.0 / s.radius
        P = (ns[k + 1] - ns[k]) * c
        M = np.array([[1.0, 0.0], [-P, 1.0]]) @ M
        if k < len(L.surfaces) - 1:
            M = np.array([[1.0, s.thickness / ns[k + 1]], [0.0, 1.0]]) @ M
    return M


@pytest.mark.parametrize("config", [1, 2])
def test_paraxial_focal_lengths(config):
    """EFL and front focal distance from finite-height traces (h = 1e-3 mm)
    agree with the ABCD system matrix to 1e-6 relative."""
    L = synth.config_lens(config)
    lam = 587.5
    M = _abcd(L, lam)
    efl = -1.0 / M[1, 0]
    # image side: parallel ray from the sensor side, h small; exit at z = 0
    h = 1e-3
    seq = oracle.build_sequence(L, 0)
    ok, p, d, _, _ = oracle.trace_sequence(L, seq, lam, (h, 0, L.sensor_z), (0, 0, -1), 0.0, -1)
    assert ok
    efl_tr = h / math.tan(math.atan2(-d[0], -d[2]))  # slope of the emerging ray
    assert abs(efl_tr - efl) / efl < 1e-6
    # front focal point: where the emerging ray crosses the axis (z < 0)
    zf_trace = p[2] - p[0] * d[2] / d[0]
    # ABCD: for light entering from the image side, the front focal distance
    # measured from the front vertex is -D/C of the matrix (vertex to vertex)
    ffd = M[1, 1] / M[1, 0]
    assert abs(zf_trace - ffd) / abs(ffd) < 1e-6
    # forward direction: a parallel ray from the object side focuses at the
    # back focal distance A/C behind the last vertex
    fwd = [(k, 2 if s.is_stop else 0, +1) for k, s in enumerate(L.surfaces)]
    zlast = L.vertex_z[-1]
    ok, p2, d2, _, _ = oracle.trace_sequence(L, fwd, lam, (h, 0, -5.0), (0, 0, 1), zlast, +1)
    assert ok
    zb = zlast - p2[0] * d2[2] / d2[0]
    bfd = -M[0, 0] / M[1, 0]
    assert abs((zb - zlast) - bfd) / abs(bfd) < 1e-6


@pytest.mark.parametrize("config", [1, 2])
def test_rotation_reflection_equivariance(config):
    """T(R p, R w) = R T(p, w) for rotations about the axis and mirror planes
    containing it (Sec. 4.1 symmetry equation)."""
    L = synth.config_lens(config)
    rng = np.random.default_rng(7)
    seqs = [oracle.build_sequence(L, 0)]
    nr = L.n_refracting
    seqs.append(oracle.build_sequence(L, 1, 1, nr))
    rays = synth.make_rays(L, 400, 99)
    checked = 0
    for seq in seqs:
        for r in range(400):
            p0 = np.array([rays["x"][r], rays["y"][r], L.sensor_z], np.float64)
            d0 = np.array([rays["dx"][r], rays["dy"][r], rays["dz"][r]], np.float64)
            lam = float(rays["lambda_nm"][r])
            ok, p, d, I, dg = oracle.trace_sequence(L, seq, lam, p0, d0, 0.0, -1)
            if not ok or dg["edge_margin"] < 1e-6:
                continue
            a = rng.uniform(0, 2 * math.pi)
            Rm = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
            if r % 2:
                Rm = Rm @ np.diag([-1.0, 1.0, 1.0])
            ok2, p2, d2, I2, _ = oracle.trace_sequence(L, seq, lam, Rm @ p0, Rm @ d0, 0.0, -1)
            assert ok2
            assert np.allclose(p2, Rm @ p, atol=1e-11, rtol=0)
            assert np.allclose(d2, Rm @ d, atol=1e-13, rtol=0)
            assert abs(I2 - I) < 1e-14
            checked += 1
    assert checked > 50


@pytest.mark.parametrize("path", [(0, 0, 0), (1, 2, 5), (1, 7, 11)])
def test_reversibility(path):
    """Tracing the exit ray back along the reversed sequence returns to the
    sensor point with the reversed input direction and the same throughput."""
    L = synth.config_lens(2)
    seq = oracle.build_sequence(L, *path)
    # a reversed transmission crosses from the other side; a reversed
    # reflection is still met from the same side
    rev = [(s, t, d if t == 1 else -d) for (s, t, d) in reversed(seq)]
    rays = synth.make_rays(L, 3000, 5)
    n = 0
    for r in range(3000):
        p0 = np.array([rays["x"][r], rays["y"][r], L.sensor_z], np.float64)
        d0 = np.array([rays["dx"][r], rays["dy"][r], rays["dz"][r]], np.float64)
        d0 /= np.linalg.norm(d0)
        lam = float(rays["lambda_nm"][r])
        ok, p, d, I, dg = oracle.trace_sequence(L, seq, lam, p0, d0, 0.0, -1)
        if not ok or dg["edge_margin"] < 1e-6:
            continue
        ok2, pb, db, Ib, _ = oracle.trace_sequence(L, rev, lam, p, -d, L.sensor_z, +1)
        assert ok2
        assert np.allclose(pb, p0, atol=1e-9, rtol=0)
        assert np.allclose(db, -d0, atol=1e-12, rtol=0)
        assert abs(Ib - I) < 1e-13 * max(1.0, I)
        n += 1
        if n >= 40:
            break
    assert n >= 10


def test_energy_bound():
    """Transmit + all two-reflection ghosts never carry more than the input."""
    L = synth.config_lens(1)
    rays = synth.make_rays(L, 5000, 11)
    tot = oracle.trace(L, rays)["throughput"].copy()
    nr = L.n_refracting
    for j in range(1, nr + 1):
        for i in range(j + 1, nr + 1):
            tot += oracle.trace(L, rays, path=(1, j, i))["throughput"]
    assert np.all(tot <= 1.0 + 1e-12)
    assert tot.max() > 0.5


# ------------------------------------------------------------ dispersion ---

def test_sellmeier_published_glass():
    """Sellmeier coefficients of a common borosilicate crown (Schott catalogue)
    give its catalogue indices n_d = 1.5168, n_F = 1.5224, n_C = 1.5143."""
    g = Glass(2, [1.03961212, 0.231792344, 1.01046945, 0.00600069867, 0.0200179144, 103.560653])
    L = Lens([Surface(0.0, 1.0, 5.0, 1, 0)], [AIR, g])
    assert abs(oracle.glass_index(L, 1, 587.5618) - 1.5168) < 5e-5
    assert abs(oracle.glass_index(L, 1, 486.1327) - 1.5224) < 5e-5
    assert abs(oracle.glass_index(L, 1, 656.2725) - 1.5143) < 5e-5


def test_cauchy_and_air():
    L = Lens([Surface(0.0, 1.0, 5.0, 1, 0)], [AIR, cauchy(1.5046, 0.00420)])
    # a two-term Cauchy fit of the same crown reproduces n_d within 1e-3
    assert abs(oracle.glass_index(L, 1, 587.56) - 1.5168) < 1e-3
    assert oracle.glass_index(L, 0, 500.0) == 1.0


@pytest.mark.parametrize("config", [1, 2])
def test_generated_glasses_normal_dispersion(config):
    L = synth.config_lens(config)
    lams = np.linspace(400, 700, 31)
    for gi in range(1, len(L.glasses)):
        ns = np.array([oracle.glass_index(L, gi, l) for l in lams])
        assert np.all(np.diff(ns) < 0) and ns.min() > 1.4


def test_serve_lenses_sellmeier_dispersion():
    for L in synth.serve_lenses()[:3]:
        for gi in range(1, len(L.glasses)):
            ns = np.array([oracle.glass_index(L, gi, l) for l in np.linspace(380, 780, 21)])
            assert np.all(np.diff(ns) < 0) and 1.45 <= ns.min() and ns.max() <= 1.95


# ---------------------------------------------------------- path lists -----

def test_ghost_sequence_structure():
    """Ghost (j,i): N + 2(i-j) interactions with exactly two reflections;
    C(N,2) distinct ghosts; the stop is a crossing, not an interaction."""
    L = synth.config_lens(2)
    N = L.n_refracting
    assert N == 11
    count = 0
    for j in range(1, N + 1):
        for i in range(j + 1, N + 1):
            seq = oracle.build_sequence(L, 1, j, i)
            inter = [s for s in seq if s[1] != 2]
            assert len(inter) == N + 2 * (i - j)
            assert sum(1 for s in inter if s[1] == 1) == 2
            count += 1
    assert count == 55
    with pytest.raises(ValueError):
        oracle.build_sequence(L, 1, 3, 3)
    with pytest.raises(ValueError):
        oracle.build_sequence(L, 1, 0, 2)
