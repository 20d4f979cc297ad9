"""Hohlraum QoIs laid out on the host (Sec. 3.2.2; layout Sec. 3.2.1): the QoI-1 probes and the
green-band QoI-3 to QoI-6.

QoI-1 averages phi, J_x and J_y over a ball of radius 0.01 around each of
four points and over each tenth of [0, T]. ``probe_cells`` gives every cell
of each ball its weight, the exact area of the cell inside the ball over the
ball's area; the plan accumulates the windows on the device (``Plan(...,
probes=probe_cells(problem))``, ``Plan.probes()``).

All four are functionals of a = sigma_a * Phi, with Phi the fluence (time
integral of the scalar flux) that a plan made with ``fluence=True``
accumulates on the device:

  QoI-3  A_G  mean over the 44 green blocks (0.05 x 0.05, counter-clockwise
              from the one centred at (-0.175, -0.375)) of the block mean A_i;
  QoI-4  V_G  mean of (A_G - A_i)^2 over the blocks;
  QoI-5  A_L  mean of a along L, the closed path through the block centres
              (the rectangle with corners (+-0.175, +-0.375), length 2.2);
  QoI-6  V_L  mean of (A_L - a)^2 along L.

This module only lays out the geometry on the host: which cells each block
and each piece of L covers, with what weight. The sums run on the device
(``Plan.fluence_functionals``). On a cell-constant field a block mean weights
each cell by its overlap area; where L runs along a face between two cells,
a on L is the mean of the two.
"""

from __future__ import annotations

import math

import numpy as np

from ._lib import FLUENCE_PIECE, PROBE_CELL

BLOCK = 0.05
# walk of the block centres: start, then (step direction, steps) per side
_START = (-0.175, -0.375)
_SIDES = [((1, 0), 7), ((0, 1), 15), ((-1, 0), 7), ((0, -1), 15)]
_EPS = 1e-9  # fraction of a cell below which a coordinate is taken to lie on a face


def block_centres() -> list[tuple[float, float]]:
    """The 44 green block centres, counter-clockwise from (-0.175, -0.375)."""
    out = []
    x, y = _START
    for (dx, dy), n in _SIDES:
        for _ in range(n):
            out.append((round(x, 12), round(y, 12)))
            x, y = x + dx * BLOCK, y + dy * BLOCK
    return out


def _span(lo: float, h: float, n: int, a: float, b: float):
    """Cells of one axis meeting [a, b] with positive length, and the lengths."""
    first = max(0, int(math.floor((a - lo) / h)))
    last = min(n, int(math.ceil((b - lo) / h)))
    idx = np.arange(first, last)
    left = lo + idx * h
    ov = np.minimum(left + h, b) - np.maximum(left, a)
    keep = ov > _EPS * h
    return idx[keep], ov[keep]


def _across(c: float, lo: float, h: float, n: int):
    """The two cells whose mean is the trace at coordinate c: the cells on
    both sides of a face, or the containing cell twice."""
    u = (c - lo) / h
    k = int(round(u))
    if abs(u - k) < _EPS:
        return min(max(k - 1, 0), n - 1), min(k, n - 1)
    k = int(math.floor(u))
    return k, k


def green_band_pieces(problem):
    """(pieces, set_start, n_blocks) for ``Plan.fluence_functionals``: the 44
    blocks as sets 0..43 (area weights), L as set 44 (length weights)."""
    nx, ny, h = problem.nx, problem.ny, problem.h
    x0, y0 = problem.x0, problem.y0
    cells_a, cells_b, weights, starts = [], [], [], [0]
    for (cx, cy) in block_centres():
        ix, lx = _span(x0, h, nx, cx - BLOCK / 2, cx + BLOCK / 2)
        jy, ly = _span(y0, h, ny, cy - BLOCK / 2, cy + BLOCK / 2)
        c = (jy[:, None] * nx + ix[None, :]).reshape(-1)
        cells_a.append(c)
        cells_b.append(c)
        weights.append((ly[:, None] * lx[None, :]).reshape(-1) / (BLOCK * BLOCK))
        starts.append(starts[-1] + c.size)
    corners = [(-0.175, -0.375), (0.175, -0.375), (0.175, 0.375), (-0.175, 0.375)]
    segs = []
    for s in range(4):
        (xa, ya), (xb, yb) = corners[s], corners[(s + 1) % 4]
        if ya == yb:  # along x at fixed y
            lo, n_along = x0, nx
            a, b = min(xa, xb), max(xa, xb)
            ja, jb = _across(ya, y0, h, ny)
            idx, ln = _span(lo, h, n_along, a, b)
            segs.append((ja * nx + idx, jb * nx + idx, ln))
        else:  # along y at fixed x
            lo, n_along = y0, ny
            a, b = min(ya, yb), max(ya, yb)
            ia, ib = _across(xa, x0, h, nx)
            idx, ln = _span(lo, h, n_along, a, b)
            segs.append((idx * nx + ia, idx * nx + ib, ln))
    length = sum(float(ln.sum()) for _, _, ln in segs)
    for ca, cb, ln in segs:
        cells_a.append(ca)
        cells_b.append(cb)
        weights.append(ln / length)
    starts.append(starts[-1] + sum(ca.size for ca, _, _ in segs))
    pieces = np.zeros(starts[-1], dtype=FLUENCE_PIECE)
    pieces["cell_a"] = np.concatenate(cells_a)
    pieces["cell_b"] = np.concatenate(cells_b)
    pieces["weight"] = np.concatenate(weights)
    return pieces, np.array(starts, dtype=np.int32), 44


def green_band_qois(plan) -> dict:
    """QoI-3 to QoI-6 of the fluence a plan has accumulated so far."""
    pieces, starts, nb = green_band_pieces(plan.problem)
    return plan.fluence_functionals(pieces, starts, nb)


PROBE_CENTRES = ((-0.4, 0.0), (0.4, 0.0), (0.0, -0.5), (0.0, 0.5))
PROBE_RADIUS = 0.01
PROBE_WINDOWS = 10


def _disc_below(x: float, y: float, r: float) -> float:
    """Area of the disc of radius r about the origin with X <= x and Y <= y.

    The disc's column at X = t spans |Y| <= s(t) = sqrt(r^2 - t^2); below
    the line Y = y it holds min(y, s) + s when that is positive. With
    a = sqrt(r^2 - y^2) that is 2s for |t| >= a and y + s for |t| < a when
    y >= 0, and y + s for |t| < a (nothing elsewhere) when y < 0. The
    integral of s is S(t) = (t s(t) + r^2 asin(t / r)) / 2.
    """
    if y <= -r or x <= -r:
        return 0.0
    x = min(x, r)

    def S(t):
        return 0.5 * (t * math.sqrt(max(r * r - t * t, 0.0)) + r * r * math.asin(max(-1.0, min(1.0, t / r))))

    if y >= r:
        return 2.0 * (S(x) - S(-r))
    a = math.sqrt(r * r - y * y)
    total = 0.0
    # middle band |t| < a: y + s
    lo, hi = -a, min(x, a)
    if hi > lo:
        total += y * (hi - lo) + S(hi) - S(lo)
    if y >= 0:  # outer bands |t| >= a: 2 s
        hi = min(x, -a)
        if hi > -r:
            total += 2.0 * (S(hi) - S(-r))
        if x > a:
            total += 2.0 * (S(x) - S(a))
    return total


def disc_rect_area(cx, cy, r, x0, x1, y0, y1) -> float:
    """Exact area of the disc about (cx, cy) inside [x0, x1] x [y0, y1]."""
    def q(x, y):
        return _disc_below(x - cx, y - cy, r)

    return max(0.0, q(x1, y1) - q(x0, y1) - q(x1, y0) + q(x0, y0))


def probe_cells(problem, centres=PROBE_CENTRES, r: float = PROBE_RADIUS, n_windows: int = PROBE_WINDOWS) -> dict:
    """The probes as ``Plan(..., probes=...)`` takes them: every cell meeting a
    ball with weight (area inside the ball) / (pi r^2)."""
    nx, ny, h = problem.nx, problem.ny, problem.h
    recs = []
    for q, (cx, cy) in enumerate(centres):
        i0 = max(0, int(math.floor((cx - r - problem.x0) / h)))
        i1 = min(nx, int(math.ceil((cx + r - problem.x0) / h)))
        j0 = max(0, int(math.floor((cy - r - problem.y0) / h)))
        j1 = min(ny, int(math.ceil((cy + r - problem.y0) / h)))
        for j in range(j0, j1):
            for i in range(i0, i1):
                xa, ya = problem.x0 + i * h, problem.y0 + j * h
                area = disc_rect_area(cx, cy, r, xa, xa + h, ya, ya + h)
                if area > _EPS * h * h:
                    recs.append((j * nx + i, q, area / (math.pi * r * r)))
    cells = np.array(recs, dtype=PROBE_CELL)
    return dict(n_probes=len(centres), n_windows=n_windows, cells=cells)


__all__ = ["block_centres", "green_band_pieces", "green_band_qois", "probe_cells", "disc_rect_area"]
