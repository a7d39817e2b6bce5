"""Path identifiers written out by walking the path (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

Sec. 3 (path-decomposition figure) identifies a light path by its sequence
of scattering decisions read as a binary number.  The paper does not fix the
bit order or whether the aperture stop is an event.  Reading used here: the
events are the refracting-surface interactions (the stop is a pass/fail
crossing, not a decision), listed in the direction light travels from the
scene to the sensor, each written as one bit (reflect = 1, transmit = 0)
after a leading 1, the first event being the most significant bit.

The walk below follows the light: it enters at surface 1 moving toward the
image, transmits until it reaches the first reflecting surface of its path,
turns around, and so on until it passes the last surface.
"""
from __future__ import annotations

from typing import List, Optional, Tuple


def events(n_refracting: int, path: Tuple[int, int, int]) -> List[str]:
    """Scene-to-sensor list of 'T' / 'R' events of a transmit path (0, 0, 0)
    or a two-reflection ghost (1, j, i): the scene-side light reflects first
    at i (the surface nearer the sensor), then at j."""
    kind, j, i = path
    if kind == 0:
        mirrors = []
    else:
        if not (1 <= j < i <= n_refracting):
            raise ValueError("invalid ghost")
        mirrors = [i, j]
    out = []
    s, step = 1, +1
    while 1 <= s <= n_refracting:
        if mirrors and s == mirrors[0]:
            out.append("R")
            mirrors.pop(0)
            step = -step
        else:
            out.append("T")
        s += step
    if mirrors or s != n_refracting + 1:
        raise ValueError("path does not reach the sensor")
    return out


def path_id(n_refracting: int, path: Tuple[int, int, int]) -> int:
    return int("1" + "".join("1" if e == "R" else "0" for e in events(n_refracting, path)), 2)


def decode_all(pid: int, max_surfaces: int = 40) -> List[Tuple[int, Tuple[int, int, int]]]:
    """Every (N, path) with N <= max_surfaces whose id is pid (brute force)."""
    hits = []
    for n in range(1, max_surfaces + 1):
        cands = [(0, 0, 0)] + [(1, j, i) for j in range(1, n + 1) for i in range(j + 1, n + 1)]
        for p in cands:
            if path_id(n, p) == pid:
                hits.append((n, p))
    return hits


def decode(n_refracting: int, pid: int) -> Optional[Tuple[int, int, int]]:
    for n, p in decode_all(pid, n_refracting):
        if n == n_refracting:
            return p
    return None
