"""Green-band QoIs of the Hohlraum benchmark (Sec. 3.2.1, QoI-3 to QoI-6).

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

from ._lib import FLUENCE_PIECE

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


__all__ = ["block_centres", "green_band_pieces", "green_band_qois"]
