"""Shared helpers for the GPU-versus-oracle parity tests (test code only)."""
import numpy as np

# Tolerances of the brute-force tracer against the FP64 oracle.
POS_TOL_MM = 1e-5        # Euclidean distance on the output plane
ANG_TOL_RAD = 1e-6       # angle between exit directions
THR_TOL = 1e-5           # absolute throughput
# Rays this close to a decision boundary may legitimately flip their mask:
EDGE_BAND_MM = 1e-6      # |h - semi_diameter| at any aperture or stop crossing
TIR_BAND = 1e-9          # |1 - eta^2 sin^2| at any refraction
GRAZE_BAND = 1e-12       # disc / B^2 of any intersection


def to_numpy(out):
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def angle(u, v):
    d = np.linalg.norm(u - v, axis=1)
    return 2.0 * np.arcsin(np.minimum(1.0, d / 2.0))


def compare_trace(gpu, ora, pos_tol=POS_TOL_MM, ang_tol=ANG_TOL_RAD, thr_tol=THR_TOL, sel=None,
                  pos_window=None):
    """Check GPU exit rays against oracle output (dicts of numpy arrays).

    ``sel`` restricts the comparison to those ray indices of ``gpu`` (the
    oracle then holds exactly those rays).  ``pos_window`` = (hx, hy)
    restricts the position check to rays whose oracle exit point lies in
    |x| <= hx, |y| <= hy: a ray that meets the output plane at a grazing
    angle lands a distance D*tan(theta) away, and its position error grows as
    D/dz^2 times the direction error, so far-off positions are not compared
    (their mask, direction and throughput still are).  Returns a stats dict;
    raises AssertionError with the details on failure."""
    g = gpu if sel is None else {k: v[sel] for k, v in gpu.items()}
    band = ((ora["edge_margin"] < EDGE_BAND_MM) | (ora["tir_margin"] < TIR_BAND)
            | (ora["graze_margin"] < GRAZE_BAND))
    gm = g["mask"].astype(bool)
    om = ora["mask"].astype(bool)
    flips = gm != om
    bad_flips = np.flatnonzero(flips & ~band)
    assert bad_flips.size == 0, (
        f"{bad_flips.size} mask mismatches outside the boundary band; first {bad_flips[:5]}, "
        f"edge margins {ora['edge_margin'][bad_flips[:5]]}")
    both = gm & om
    stats = {"n": int(gm.size), "valid": int(both.sum()), "band_flips": int(flips.sum()),
             "band": int(band.sum())}
    # invalid rays carry NaN fields and zero throughput
    inv = ~gm
    assert np.all(np.isnan(g["x"][inv])) and np.all(g["throughput"][inv] == 0)
    if both.any():
        pw = both
        if pos_window is not None:
            pw = both & (np.abs(ora["x"]) <= pos_window[0]) & (np.abs(ora["y"]) <= pos_window[1])
            stats["pos_compared"] = int(pw.sum())
        pos = np.hypot(g["x"][pw] - ora["x"][pw], g["y"][pw] - ora["y"][pw])
        if pos.size == 0:
            pos = np.zeros(1)
        u = np.stack([g["dx"][both], g["dy"][both], g["dz"][both]], 1).astype(np.float64)
        v = np.stack([ora["dx"][both], ora["dy"][both], ora["dz"][both]], 1)
        ang = angle(u, v)
        thr = np.abs(g["throughput"][both] - ora["throughput"][both])
        stats.update(pos_max=float(pos.max()), ang_max=float(ang.max()), thr_max=float(thr.max()))
        assert pos.max() <= pos_tol, f"exit position error {pos.max():.3e} mm > {pos_tol}"
        assert ang.max() <= ang_tol, f"exit direction error {ang.max():.3e} rad > {ang_tol}"
        assert thr.max() <= thr_tol, f"throughput error {thr.max():.3e} > {thr_tol}"
    return stats
