"""Seeded synthetic inputs: lens prescriptions and sensor-side ray batches.

This module is shared by the FP64 oracle, the HIP path's tests and the
benchmark.  It only *makes inputs*; it holds none of the per-ray arithmetic
that either side computes (no exact ray-surface intersection, refraction,
Fresnel factors or network evaluation).  To shape realistic prescriptions it
uses first-order (paraxial, thin-lens) design relations at the d-line; those
numbers only decide the prescription and are never used as expected values.

Conventions (shared by every consumer of these inputs):
  * the optical axis is z; surfaces are listed object side first, the first
    vertex sits at z = 0 and vertex k+1 at z_k + thickness_k; the sensor plane
    is at z_N + thickness_N;
  * radius > 0 puts the centre of curvature on the image side, radius 0 is flat;
  * ``glass_after`` indexes ``glasses`` and names the medium on the image side
    of the surface; index 0 is air (n = 1 exactly); object side of surface 1 is
    air;
  * the aperture stop is a flat surface with ``is_stop = 1`` and the same
    medium on both sides;
  * Cauchy glasses: n = A + B/l^2 + C/l^4, Sellmeier glasses:
    n^2 = 1 + sum_i B_i l^2/(l^2 - C_i), with l in micrometres;
  * rays start on the sensor plane travelling toward the object (dz < 0);
    wavelengths are in nanometres.

The paper's lens files are not available; the topologies below (cemented
doublet, double-Gauss-style 11-surface lens, mixed lenses of 4..22 surfaces)
are drawn from a seed following common first-order design rules (thin-lens
powers and shape factors, f/2.8 marginal ray, full-frame chief ray).
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import List, Sequence

import numpy as np

GLASS_AIR = 0
GLASS_CAUCHY = 1
GLASS_SELLMEIER = 2

LAMBDA_D_UM = 0.5875618
LAMBDA_F_UM = 0.4861327
LAMBDA_C_UM = 0.6562725

SENSOR_HALF_W = 18.0  # 36 x 24 mm frame
SENSOR_HALF_H = 12.0
SENSOR_HALF_DIAG = math.hypot(SENSOR_HALF_W, SENSOR_HALF_H)
F_NUMBER = 2.8


@dataclasses.dataclass
class Glass:
    kind: int
    coef: List[float]  # six numbers; meaning depends on kind

    def to_json(self):
        return {"kind": int(self.kind), "coef": [float(c) for c in self.coef]}


@dataclasses.dataclass
class Surface:
    radius: float
    thickness: float
    semi_diameter: float
    glass_after: int
    is_stop: int = 0

    def to_json(self):
        return dataclasses.asdict(self)


@dataclasses.dataclass
class Lens:
    surfaces: List[Surface]
    glasses: List[Glass]
    name: str = ""

    @property
    def n_surfaces(self) -> int:
        return len(self.surfaces)

    @property
    def n_refracting(self) -> int:
        return sum(1 for s in self.surfaces if not s.is_stop)

    @property
    def vertex_z(self) -> np.ndarray:
        z = [0.0]
        for s in self.surfaces[:-1]:
            z.append(z[-1] + s.thickness)
        return np.array(z)

    @property
    def sensor_z(self) -> float:
        return float(self.vertex_z[-1] + self.surfaces[-1].thickness)

    def to_json(self) -> str:
        return json.dumps({"name": self.name,
                           "surfaces": [s.to_json() for s in self.surfaces],
                           "glasses": [g.to_json() for g in self.glasses]})

    @staticmethod
    def from_json(text: str) -> "Lens":
        d = json.loads(text)
        return Lens([Surface(**s) for s in d["surfaces"]],
                    [Glass(g["kind"], list(g["coef"])) for g in d["glasses"]],
                    d.get("name", ""))

    def surface_array(self) -> np.ndarray:
        """(n_surf, 5) float64: radius, thickness, semi_diameter, glass_after, is_stop."""
        return np.array([[s.radius, s.thickness, s.semi_diameter, s.glass_after, s.is_stop]
                         for s in self.surfaces], dtype=np.float64)

    def glass_array(self) -> np.ndarray:
        """(n_glass, 7) float64: kind, coef[0..5]."""
        return np.array([[g.kind] + list(g.coef) for g in self.glasses], dtype=np.float64)


# ---------------------------------------------------------------------------
# glasses (design-time only: coefficients are derived from n_d and Abbe V_d)
# ---------------------------------------------------------------------------

def _cauchy_from_nd_vd(nd: float, vd: float) -> Glass:
    """Two-term Cauchy glass whose d-line index is nd and Abbe number vd."""
    b = (nd - 1.0) / (vd * (1.0 / LAMBDA_F_UM ** 2 - 1.0 / LAMBDA_C_UM ** 2))
    a = nd - b / LAMBDA_D_UM ** 2
    return Glass(GLASS_CAUCHY, [a, b, 0.0, 0.0, 0.0, 0.0])


def _sellmeier_index_design(g: Glass, lam_um: float) -> float:
    l2 = lam_um * lam_um
    s = 1.0
    for b, c in zip(g.coef[:3], g.coef[3:]):
        s += b * l2 / (l2 - c)
    return math.sqrt(s)


def _sellmeier_from_nd(rng: np.random.Generator, nd: float) -> Glass:
    """Three-term Sellmeier glass with d-line index nd (B1 solved for it)."""
    for _ in range(100):
        c1 = rng.uniform(0.004, 0.014)
        c2 = rng.uniform(0.02, 0.06)
        c3 = rng.uniform(90.0, 160.0)
        b2 = rng.uniform(0.05, 0.35)
        b3 = rng.uniform(0.6, 1.3)
        l2 = LAMBDA_D_UM ** 2
        rest = nd * nd - 1.0 - b2 * l2 / (l2 - c2) - b3 * l2 / (l2 - c3)
        b1 = rest * (l2 - c1) / l2
        if b1 <= 0.2:
            continue
        g = Glass(GLASS_SELLMEIER, [b1, b2, b3, c1, c2, c3])
        lams = np.linspace(0.38, 0.78, 41)
        ns = np.array([_sellmeier_index_design(g, l) for l in lams])
        if ns.min() >= 1.45 and ns.max() <= 1.95 and np.all(np.diff(ns) < 0):
            return g
    raise RuntimeError("could not draw a Sellmeier glass")


def _index_d(g: Glass) -> float:
    if g.kind == GLASS_AIR:
        return 1.0
    if g.kind == GLASS_CAUCHY:
        return g.coef[0] + g.coef[1] / LAMBDA_D_UM ** 2 + g.coef[2] / LAMBDA_D_UM ** 4
    return _sellmeier_index_design(g, LAMBDA_D_UM)


def _draw_glass(rng: np.random.Generator, flint: bool, sellmeier: bool) -> Glass:
    if flint:
        nd = rng.uniform(1.60, 1.78)
        vd = rng.uniform(25.0, 36.0)
    else:
        nd = rng.uniform(1.50, 1.70)
        vd = rng.uniform(48.0, 64.0)
    if sellmeier:
        return _sellmeier_from_nd(rng, nd)
    return _cauchy_from_nd_vd(nd, vd)


# ---------------------------------------------------------------------------
# first-order layout
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class _Elem:
    kind: str                 # "single", "cemented", "stop"
    phis: Sequence[float]     # thin-lens powers (1/mm) of the component lenses
    shape: float              # shape factor of the first component
    thick: Sequence[float]    # centre thicknesses of the components
    glasses: Sequence[int]    # glass indices of the components
    gap_after: float          # air gap to the next element


def _curvatures(elems: List[_Elem], glasses: List[Glass]):
    """Curvatures, thicknesses, glass_after and stop flags from thin-lens data."""
    rad, th, ga, st = [], [], [], []
    for e in elems:
        if e.kind == "stop":
            rad.append(0.0)
            th.append(e.gap_after)
            ga.append(GLASS_AIR)
            st.append(1)
            continue
        n0 = _index_d(glasses[e.glasses[0]])
        c1 = e.phis[0] * (e.shape + 1.0) / (2.0 * (n0 - 1.0))
        c2 = e.phis[0] * (e.shape - 1.0) / (2.0 * (n0 - 1.0))
        cs = [c1, c2]
        for k in range(1, len(e.phis)):
            nk = _index_d(glasses[e.glasses[k]])
            cs.append(cs[-1] - e.phis[k] / (nk - 1.0))
        for k, c in enumerate(cs):
            rad.append(0.0 if c == 0.0 else 1.0 / c)
            if k < len(e.phis):
                th.append(e.thick[k])
                ga.append(e.glasses[k])
            else:
                th.append(e.gap_after)
                ga.append(GLASS_AIR)
            st.append(0)
    return rad, th, ga, st


def _paraxial(rad, th, ga, st, glasses, y0, u0):
    """Paraxial y-nu trace at the d-line; returns heights at each surface and final angle."""
    n = 1.0
    y, u = y0, u0
    ys = []
    for k in range(len(rad)):
        ys.append(y)
        n2 = _index_d(glasses[ga[k]])
        c = 0.0 if rad[k] == 0.0 else 1.0 / rad[k]
        u = (n * u - y * (n2 - n) * c) / n2
        n = n2
        if k < len(rad) - 1:
            y = y + th[k] * u
    return np.array(ys), y, u


def _sag(c: float, h: float) -> float:
    if c == 0.0:
        return 0.0
    return c * h * h / (1.0 + math.sqrt(max(0.0, 1.0 - c * c * h * h)))


def _finish(rng, elems, glasses, efl_target, name, rear_sd_scale=1.1):
    """Scale to the target EFL, place the sensor at the paraxial focus, size apertures."""
    for _it in range(8):
        rad, th, ga, st = _curvatures(elems, glasses)
        _, _, u = _paraxial(rad, th, ga, st, glasses, 1.0, 0.0)
        if u >= 0:
            return None
        efl = -1.0 / u
        s = efl_target / efl
        rad = [r * s for r in rad]
        th = [t * s for t in th]
        ys, yl, ul = _paraxial(rad, th, ga, st, glasses, 1.0, 0.0)
        bfl = -yl / ul
        if not (8.0 <= bfl <= 3.0 * efl_target):
            return None
        th[-1] = bfl
        # marginal ray at f/2.8 from infinity, chief ray through the stop centre
        epd_half = efl_target / (2.0 * F_NUMBER)
        ym, _, _ = _paraxial(rad, th, ga, st, glasses, epd_half, 0.0)
        istop = st.index(1)
        ya, _, _ = _paraxial(rad, th, ga, st, glasses, 1.0, 0.0)
        yb, _, _ = _paraxial(rad, th, ga, st, glasses, 0.0, 1.0)
        u_field = SENSOR_HALF_DIAG / efl_target
        a = -u_field * yb[istop] / ya[istop]
        yc, _, _ = _paraxial(rad, th, ga, st, glasses, a, u_field)
        sd = []
        for k in range(len(rad)):
            if st[k]:
                sd.append(abs(ym[k]))
            else:
                v = rear_sd_scale * (abs(ym[k]) + abs(yc[k]))
                if rad[k] != 0.0:
                    v = min(v, 0.9 * abs(rad[k]))
                sd.append(v)
        # edge thickness / rim clearance; grow centre thickness where violated
        grew = False
        for k in range(len(rad) - 1):
            h = max(sd[k], sd[k + 1])
            c1 = 0.0 if rad[k] == 0.0 else 1.0 / rad[k]
            c2 = 0.0 if rad[k + 1] == 0.0 else 1.0 / rad[k + 1]
            hk = min(h, 0.999 / abs(c1)) if c1 else h
            hk1 = min(h, 0.999 / abs(c2)) if c2 else h
            edge = th[k] + _sag(c2, hk1) - _sag(c1, hk)
            need = 0.5 if ga[k] != GLASS_AIR else 0.3
            if edge < need:
                grew = True
                _grow(elems, k, (need - edge) / s + 0.05 / s)
        if not grew:
            surfs = [Surface(float(rad[k]), float(th[k]), float(sd[k]), int(ga[k]), int(st[k]))
                     for k in range(len(rad))]
            return Lens(surfs, glasses, name)
    return None


def _grow(elems: List[_Elem], surf_index: int, amount: float):
    """Add ``amount`` to the thickness (or gap) that follows surface ``surf_index``."""
    k = 0
    for e in elems:
        if e.kind == "stop":
            if k == surf_index:
                e.gap_after += amount
                return
            k += 1
            continue
        nsurf = len(e.phis) + 1
        if surf_index < k + nsurf:
            local = surf_index - k
            if local < len(e.phis):
                t = list(e.thick)
                t[local] += amount
                e.thick = t
            else:
                e.gap_after += amount
            return
        k += nsurf


def _double_gauss(rng: np.random.Generator, efl: float, name: str) -> Lens:
    f = 50.0
    glasses = [Glass(GLASS_AIR, [0.0] * 6)]

    def g(flint):
        glasses.append(_draw_glass(rng, flint, False))
        return len(glasses) - 1

    elems = [
        _Elem("single", [rng.uniform(0.45, 0.75) / f], rng.uniform(1.4, 2.6),
              [rng.uniform(4.0, 6.0)], [g(False)], rng.uniform(0.4, 1.5)),
        _Elem("cemented", [rng.uniform(0.55, 0.85) / f, -rng.uniform(0.9, 1.3) / f],
              rng.uniform(1.3, 2.4), [rng.uniform(5.5, 8.0), rng.uniform(1.5, 2.5)],
              [g(False), g(True)], rng.uniform(3.5, 6.0)),
        _Elem("stop", [], 0.0, [], [], rng.uniform(3.5, 6.0)),
        _Elem("single", [-rng.uniform(0.45, 0.75) / f], rng.uniform(1.6, 2.8),
              [rng.uniform(1.5, 2.8)], [g(True)], rng.uniform(0.4, 1.5)),
        _Elem("single", [rng.uniform(0.55, 0.85) / f], rng.uniform(-1.6, -0.4),
              [rng.uniform(4.0, 6.5)], [g(False)], rng.uniform(0.3, 1.2)),
        _Elem("single", [rng.uniform(0.30, 0.55) / f], rng.uniform(-1.0, 0.6),
              [rng.uniform(3.0, 5.0)], [g(False)], 0.0),
    ]
    return _finish(rng, elems, glasses, efl, name)


def _doublet(rng: np.random.Generator, efl: float, name: str) -> Lens:
    f = efl
    glasses = [Glass(GLASS_AIR, [0.0] * 6)]
    glasses.append(_draw_glass(rng, False, False))
    glasses.append(_draw_glass(rng, True, False))
    elems = [
        _Elem("stop", [], 0.0, [], [], rng.uniform(2.0, 5.0)),
        _Elem("cemented", [rng.uniform(1.9, 2.4) / f, -rng.uniform(0.9, 1.3) / f],
              rng.uniform(-0.3, 0.3), [rng.uniform(5.0, 8.0), rng.uniform(2.0, 3.5)],
              [1, 2], 0.0),
    ]
    return _finish(rng, elems, glasses, efl, name)


def _mixed(rng: np.random.Generator, n_refr: int, efl: float, name: str,
           sellmeier_frac: float = 0.5) -> Lens:
    f = 50.0
    choices = [d for d in range(0, n_refr // 3 + 1) if (n_refr - 3 * d) % 2 == 0
               and (n_refr - 3 * d) >= 0]
    n_dbl = int(rng.choice(choices))
    n_sgl = (n_refr - 3 * n_dbl) // 2
    kinds = ["cemented"] * n_dbl + ["single"] * n_sgl
    rng.shuffle(kinds)
    glasses = [Glass(GLASS_AIR, [0.0] * 6)]

    def g(flint):
        glasses.append(_draw_glass(rng, flint, rng.uniform() < sellmeier_frac))
        return len(glasses) - 1

    m = len(kinds)
    scale = 1.0 / max(1.0, 0.5 * m)
    elems: List[_Elem] = []
    for ei, k in enumerate(kinds):
        neg = (ei % 3 == 1)
        if k == "single":
            phi = (-1.0 if neg else 1.0) * rng.uniform(0.5, 1.0) * scale / f
            if neg:
                phi *= 0.8
            elems.append(_Elem("single", [phi], rng.uniform(-1.5, 1.5),
                               [rng.uniform(2.0, 5.0)], [g(neg)], rng.uniform(0.5, 2.5)))
        else:
            pa = rng.uniform(0.9, 1.5) * scale / f
            pb = -rng.uniform(0.5, 0.9) * scale / f
            elems.append(_Elem("cemented", [pa, pb], rng.uniform(-1.0, 1.0),
                               [rng.uniform(3.0, 6.0), rng.uniform(1.5, 2.5)], [g(False), g(True)],
                               rng.uniform(0.5, 2.5)))
        if ei == (m - 1) // 2:
            elems.append(_Elem("stop", [], 0.0, [], [], rng.uniform(2.0, 4.0)))
    elems[-1].gap_after = 0.0
    return _finish(rng, elems, glasses, efl, name)


def make_lens(kind: str, seed: int, n_refracting: int = 11, efl: float | None = None) -> Lens:
    """Draw a prescription of the given topology from ``seed`` (PCG64).

    kind: "doublet" (3 surfaces + front stop, EFL 50-100 mm), "double_gauss"
    (11 surfaces + stop, EFL 50 mm) or "mixed" (``n_refracting`` surfaces,
    Cauchy and Sellmeier glasses, EFL 50 mm).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    for attempt in range(200):
        if kind == "doublet":
            lens = _doublet(rng, efl or float(rng.uniform(50.0, 100.0)), f"doublet-s{seed}")
        elif kind == "double_gauss":
            lens = _double_gauss(rng, efl or 50.0, f"double-gauss-s{seed}")
        elif kind == "mixed":
            lens = _mixed(rng, n_refracting, efl or 50.0, f"mixed{n_refracting}-s{seed}")
        else:
            raise ValueError(kind)
        if lens is not None and _sane(lens):
            return lens
    raise RuntimeError(f"no valid {kind} lens from seed {seed}")


def _sane(lens: Lens) -> bool:
    for s in lens.surfaces:
        if s.semi_diameter <= 0 or s.thickness < 0:
            return False
        if s.radius != 0.0 and s.semi_diameter >= abs(s.radius):
            return False
    return sum(s.is_stop for s in lens.surfaces) == 1


# ---------------------------------------------------------------------------
# sensor-side rays
# ---------------------------------------------------------------------------

def make_rays(lens: Lens, n: int, seed: int, lam_range=(400.0, 700.0)) -> dict:
    """n sensor-side rays as float32 SoA arrays (x, y, dx, dy, dz, lambda_nm).

    Sensor point uniform on the 36 x 24 mm frame; target point uniform by area
    on the disk of the last surface's semi-diameter in its vertex plane;
    direction = normalised (target - sensor point) in float64, then rounded to
    float32; wavelength uniform in ``lam_range`` nm.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-SENSOR_HALF_W, SENSOR_HALF_W, n)
    y = rng.uniform(-SENSOR_HALF_H, SENSOR_HALF_H, n)
    u1 = rng.uniform(0.0, 1.0, n)
    u2 = rng.uniform(0.0, 1.0, n)
    lam = rng.uniform(lam_range[0], lam_range[1], n)
    rear = lens.surfaces[-1]
    rho = rear.semi_diameter * np.sqrt(u1)
    phi = 2.0 * np.pi * u2
    tx = rho * np.cos(phi)
    ty = rho * np.sin(phi)
    tz = -rear.thickness  # rear vertex plane relative to the sensor plane
    vx, vy = tx - x, ty - y
    vz = np.full(n, tz)
    norm = np.sqrt(vx * vx + vy * vy + vz * vz)
    f32 = np.float32
    return {"x": x.astype(f32), "y": y.astype(f32),
            "dx": (vx / norm).astype(f32), "dy": (vy / norm).astype(f32),
            "dz": (vz / norm).astype(f32), "lambda_nm": lam.astype(f32)}


def make_forward_rays(lens: Lens, n: int, seed: int, half_angle_deg: float = 20.0, direction=None,
                      aperture_scale: float = 1.1, lam_range=(400.0, 700.0)) -> dict:
    """n scene-side rays for forward light tracing, as float32 SoA arrays.

    The start point is uniform by area on a disk of aperture_scale times the
    first surface's semi-diameter (in the forward input plane).  The direction
    is either the given unit vector (a distant point light) or uniform in
    solid angle within half_angle_deg of the axis, travelling toward the
    image.  The wavelength is uniform in lam_range nm."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r0 = aperture_scale * lens.surfaces[0].semi_diameter
    rho = r0 * np.sqrt(rng.uniform(0.0, 1.0, n))
    phi = 2.0 * np.pi * rng.uniform(0.0, 1.0, n)
    if direction is None:
        cmin = math.cos(math.radians(half_angle_deg))
        cz = rng.uniform(cmin, 1.0, n)
        az = 2.0 * np.pi * rng.uniform(0.0, 1.0, n)
        sz = np.sqrt(1.0 - cz * cz)
        d = np.stack([sz * np.cos(az), sz * np.sin(az), cz], 1)
    else:
        d = np.tile(np.asarray(direction, np.float64) / np.linalg.norm(direction), (n, 1))
        rng.uniform(0.0, 1.0, 2 * n)   # keep the stream aligned with the cone case
    lam = rng.uniform(lam_range[0], lam_range[1], n)
    f32 = np.float32
    return {"x": (rho * np.cos(phi)).astype(f32), "y": (rho * np.sin(phi)).astype(f32),
            "dx": d[:, 0].astype(f32), "dy": d[:, 1].astype(f32), "dz": d[:, 2].astype(f32),
            "lambda_nm": lam.astype(f32)}


RAY_FIELDS = ("x", "y", "dx", "dy", "dz", "lambda_nm")

# workload presets ---------------------------------------------------------
# C1: cemented doublet + stop, 65,536 rays.  C2: 11-surface double-Gauss-style
# lens, 4,194,304 rays.  C3: same lens, 16,777,216 rays.  C4: same lens,
# training.  C5: eight mixed lenses with 4..22 refracting surfaces.
SERVE_SURFACES = (4, 6, 8, 11, 13, 16, 19, 22)


def config_lens(config: int) -> Lens:
    if config == 1:
        return make_lens("doublet", 1000 + config)
    if config in (2, 3, 4):
        return make_lens("double_gauss", 1000 + 2)
    raise ValueError(config)


def serve_lenses() -> List[Lens]:
    return [make_lens("mixed", 1005 * 10 + i, n_refracting=k) for i, k in enumerate(SERVE_SURFACES)]


def config_rays(config: int, n: int | None = None) -> dict:
    sizes = {1: 65536, 2: 4194304, 3: 16777216, 4: 65536}
    lens = config_lens(config)
    return make_rays(lens, sizes[config] if n is None else n, 2000 + config)


# counter-based ray generator (host twin of the device generator) ----------
# Philox4x64-10 from its published definition (Salmon, Moraes, Dror and Shaw,
# SC 2011): ten rounds of two 64x64->128-bit multiplies with the Weyl key
# schedule.  Ray k uses counter (first + k, 0, 0, 0) and key (seed, 0).

_M32 = np.uint64(0xFFFFFFFF)
_PH_M = (np.uint64(0xD2E7470EE14C6C93), np.uint64(0xCA5A826395121157))
_PH_W = (np.uint64(0x9E3779B97F4A7C15), np.uint64(0xBB67AE8584CAA73B))


def _mulhilo64(a, b):
    a = np.asarray(a, np.uint64)
    b = np.asarray(b, np.uint64)
    s32 = np.uint64(32)
    a0, a1 = a & _M32, a >> s32
    b0, b1 = b & _M32, b >> s32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> s32) + (p01 & _M32) + (p10 & _M32)
    return p11 + (p01 >> s32) + (p10 >> s32) + (mid >> s32), a * b


def philox4x64_10(ctr, key):
    """Philox4x64-10 of counter words ctr[0..3] (arrays) and key (k0, k1)."""
    x0, x1, x2, x3 = (np.asarray(c, np.uint64).copy() for c in ctr)
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo64(_PH_M[0], x0)
            hi1, lo1 = _mulhilo64(_PH_M[1], x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + _PH_W[0]
            k1 = k1 + _PH_W[1]
    return x0, x1, x2, x3


def philox_rays(lens: Lens, n: int, seed: int, first: int = 0, half_w: float = SENSOR_HALF_W,
                half_h: float = SENSOR_HALF_H, lam_range=(400.0, 700.0)) -> dict:
    """Rays k = 0..n-1 of the counter-based generator, computed in float64
    from the same 24-bit uniforms and rounded to float32 (the sensor point is
    rounded before the direction is formed, as on the device)."""
    ctr = np.arange(n, dtype=np.uint64) + np.uint64(first)
    z = np.zeros(n, np.uint64)
    o0, o1, o2, o3 = philox4x64_10((ctr, z, z, z), (seed, 0))
    s40, s16, m24 = np.uint64(40), np.uint64(16), np.uint64(0xFFFFFF)
    u0, u1, u2, u3 = ((o >> s40).astype(np.float64) * 2.0 ** -24 for o in (o0, o1, o2, o3))
    u4 = ((o0 >> s16) & m24).astype(np.float64) * 2.0 ** -24
    return rays_from_uniforms(lens, np.stack([u0, u1, u2, u3, u4]), half_w, half_h, lam_range)


def rays_from_uniforms(lens: Lens, u: np.ndarray, half_w: float = SENSOR_HALF_W,
                       half_h: float = SENSOR_HALF_H, lam_range=(400.0, 700.0),
                       lam: np.ndarray | None = None) -> dict:
    """Sensor-side rays of points u (5, n) of [0, 1)^5: sensor point
    (2 u0 - 1) * half extents, target point on the rear disk at radius
    sd * sqrt(u2) and angle 2 pi u3, wavelength lambda_min + u4 * range (or
    the given wavelengths).  Float64 from the given values, rounded to
    float32 (the sensor point before the direction is formed, as on the
    device)."""
    u = np.asarray(u, np.float64)
    n = u.shape[1]
    f32 = np.float32
    hw, hh = float(f32(half_w)), float(f32(half_h))
    sx = (2.0 * hw * u[0] - hw).astype(f32)
    sy = (2.0 * hh * u[1] - hh).astype(f32)
    rear = lens.surfaces[-1]
    rho = float(f32(rear.semi_diameter)) * np.sqrt(u[2])
    phi = 2.0 * np.pi * u[3]
    vx = rho * np.cos(phi) - sx.astype(np.float64)
    vy = rho * np.sin(phi) - sy.astype(np.float64)
    vz = np.full(n, -float(f32(rear.thickness)))
    norm = np.sqrt(vx * vx + vy * vy + vz * vz)
    l0, l1 = float(f32(lam_range[0])), float(f32(lam_range[1]))
    lam_out = ((l1 - l0) * u[4] + l0).astype(f32) if lam is None else np.asarray(lam, f32)
    return {"x": sx, "y": sy, "dx": (vx / norm).astype(f32), "dy": (vy / norm).astype(f32),
            "dz": (vz / norm).astype(f32), "lambda_nm": lam_out}


def philox_forward_rays(n: int, seed: int, light=(0.0, 0.0, 1.0), at_infinity: bool = True,
                        aperture: float = 1.0, z_plane: float = 0.0, first: int = 0,
                        lam_range=(400.0, 700.0)) -> dict:
    """Host twin of the device's forward generator: rays k = 0..n-1 from a
    point light, p_in uniform by area on the aperture disk (float64 from the
    same 24-bit uniforms, rounded to float32), direction the light's
    (at infinity) or normalised p_in - light with p_in on the plane z_plane."""
    ctr = np.arange(n, dtype=np.uint64) + np.uint64(first)
    z = np.zeros(n, np.uint64)
    o0, o1, o2, _ = philox4x64_10((ctr, z, z, z), (seed, 0))
    s40 = np.uint64(40)
    u0, u1, u2 = ((o >> s40).astype(np.float64) * 2.0 ** -24 for o in (o0, o1, o2))
    f32 = np.float32
    rho = float(f32(aperture)) * np.sqrt(u0)
    phi = 2.0 * np.pi * u1
    px = (rho * np.cos(phi)).astype(f32)
    py = (rho * np.sin(phi)).astype(f32)
    if at_infinity:
        v = np.asarray(light, np.float32).astype(np.float64)   # the device receives FP32
        d = np.tile(v / np.linalg.norm(v), (n, 1))
    else:
        lx, ly, lz = (float(f32(c)) for c in light)
        d = np.stack([px.astype(np.float64) - lx, py.astype(np.float64) - ly,
                      np.full(n, float(f32(z_plane)) - lz)], 1)
        d /= np.linalg.norm(d, axis=1, keepdims=True)
    l0, l1 = float(f32(lam_range[0])), float(f32(lam_range[1]))
    return {"x": px, "y": py, "dx": d[:, 0].astype(f32), "dy": d[:, 1].astype(f32),
            "dz": d[:, 2].astype(f32), "lambda_nm": ((l1 - l0) * u2 + l0).astype(f32)}
