"""Hohlraum QoI-1 probes and QoI-3 to QoI-6 from a fluence field (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the parity tests and
the script that writes the stored expected values use it; the product path
never does.

The fluence is the time integral of the scalar flux per cell, Phi = int_0^T
phi dt (``oracle.solve(..., fluence=True)``); the discrete solution is constant
on each cell. The four QoIs of the Hohlraum benchmark (Sec. 3.2.2) integrate
a(x, y) = sigma_a(x, y) Phi(x, y) over the green capsule band:

  QoI-3  A_G = (1/N_G) sum_i A_i, with A_i the mean of a over green block g_i
         (N_G = 44 blocks of 0.05 x 0.05, numbered counter-clockwise from the
         block centred at (-0.175, -0.375));
  QoI-4  V_G = (1/N_G) sum_i |A_G - A_i|^2;
  QoI-5  A_L = (1/length(L)) int_L a ds, L the closed path through the block
         centres (the rectangle with corners (+-0.175, +-0.375), length 2.2);
  QoI-6  V_L = (1/length(L)) int_L |A_L - a|^2 ds.

QoI-1 averages phi, J_x and J_y over a ball B_r (r = 0.01) around each of
four probe points and over each tenth of [0, T], divided by the space-time
volume |B_r| T/10 (``probe_cells`` gives each cell's weight, the area of the
cell inside the ball over |B_r|; the oracle's stepping does the rest).

Readings where the paper is silent: a block mean weights every cell by the
area it shares with the block (exact for the cell-constant solution); where
L runs along a cell face, a on L is the mean of the two cells that share the
face (the two one-sided traces weighted equally); sigma_a is the cell's own
(region) value. The code is plain loops over blocks, segments and cells.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import integrate

BLOCK = 0.05
N_BLOCKS = 44
# corners of L, counter-clockwise from the first block's centre
LINE_CORNERS = [(-0.175, -0.375), (0.175, -0.375), (0.175, 0.375), (-0.175, 0.375)]


def green_block_centres():
    """Centres of the 44 green blocks, counter-clockwise from (-0.175, -0.375).

    The band is the ring of 0.05 blocks between (-0.20, 0.20) x (-0.40, 0.40)
    and (-0.15, 0.15) x (-0.35, 0.35): its block centres lie on L, 0.05 apart.
    Walking L from its first corner in steps of 0.05 visits every centre once.
    """
    centres = []
    for c in range(4):
        (xa, ya), (xb, yb) = LINE_CORNERS[c], LINE_CORNERS[(c + 1) % 4]
        n = int(round(math.hypot(xb - xa, yb - ya) / BLOCK))
        for s in range(n):  # the far corner starts the next side
            centres.append((xa + (xb - xa) * s / n, ya + (yb - ya) * s / n))
    return centres


def _cell_value(p, fluence, i, j):
    return float(p.sigma_a[p.region[j, i]]) * float(fluence[j, i])


def block_means(p, fluence):
    """A_i for the 44 blocks: area-weighted mean of sigma_a * Phi."""
    out = []
    for (cx, cy) in green_block_centres():
        bx0, bx1 = cx - BLOCK / 2, cx + BLOCK / 2
        by0, by1 = cy - BLOCK / 2, cy + BLOCK / 2
        total = 0.0
        for j in range(p.ny):
            y0, y1 = p.y0 + j * p.h, p.y0 + (j + 1) * p.h
            oy = min(y1, by1) - max(y0, by0)
            if oy <= 1e-9 * p.h:  # disjoint, or sharing only an edge up to rounding
                continue
            for i in range(p.nx):
                x0, x1 = p.x0 + i * p.h, p.x0 + (i + 1) * p.h
                ox = min(x1, bx1) - max(x0, bx0)
                if ox <= 1e-9 * p.h:
                    continue
                total += ox * oy * _cell_value(p, fluence, i, j)
        out.append(total / (BLOCK * BLOCK))
    return np.array(out)


def _cells_at(coord, lo, h, n):
    """Cells whose closed extent holds ``coord`` along one axis: one cell, or
    the two that share a face when ``coord`` lies on it (to 1e-9 of a cell)."""
    u = (coord - lo) / h
    k = round(u)
    if abs(u - k) < 1e-9:
        return [c for c in (k - 1, k) if 0 <= c < n]
    return [int(math.floor(u))]


def line_pieces(p):
    """L cut at every grid line it crosses: a list of (length, [(i, j), ...])
    with the cells whose mean gives a on that piece."""
    pieces = []
    for c in range(4):
        (xa, ya), (xb, yb) = LINE_CORNERS[c], LINE_CORNERS[(c + 1) % 4]
        horizontal = ya == yb
        a0, a1 = (xa, xb) if horizontal else (ya, yb)
        lo = p.x0 if horizontal else p.y0
        n_along = p.nx if horizontal else p.ny
        # breakpoints: the ends and every face strictly between them
        s0, s1 = min(a0, a1), max(a0, a1)
        cuts = [s0, s1]
        k0 = math.floor((s0 - lo) / p.h) + 1
        k1 = math.ceil((s1 - lo) / p.h) - 1
        for k in range(k0, k1 + 1):
            f = lo + k * p.h
            if s0 + 1e-12 < f < s1 - 1e-12:
                cuts.append(f)
        cuts.sort()
        fixed = ya if horizontal else xa
        across = _cells_at(fixed, p.y0 if horizontal else p.x0, p.h, p.ny if horizontal else p.nx)
        for q in range(len(cuts) - 1):
            mid = 0.5 * (cuts[q] + cuts[q + 1])
            along = _cells_at(mid, lo, p.h, n_along)
            cells = [(a, b) if horizontal else (b, a) for a in along for b in across]
            pieces.append((cuts[q + 1] - cuts[q], cells))
    return pieces


def qois(p, fluence):
    """Dict with A_G, V_G, A_L, V_L (QoI-3 to QoI-6), the 44 A_i and the
    length of L."""
    A = block_means(p, fluence)
    A_G = float(sum(A) / len(A))
    V_G = float(sum((A_G - a) ** 2 for a in A) / len(A))
    pieces = line_pieces(p)
    length = sum(d for d, _ in pieces)
    vals = [(d, sum(_cell_value(p, fluence, i, j) for i, j in cells) / len(cells)) for d, cells in pieces]
    A_L = sum(d * v for d, v in vals) / length
    V_L = sum(d * (A_L - v) ** 2 for d, v in vals) / length
    return dict(A_G=A_G, V_G=V_G, A_L=float(A_L), V_L=float(V_L), A=A, length=length)


PROBE_CENTRES = [(-0.4, 0.0), (0.4, 0.0), (0.0, -0.5), (0.0, 0.5)]
PROBE_RADIUS = 0.01
N_WINDOWS = 10


def disc_cell_area(cx, cy, r, x0, x1, y0, y1):
    """Area of the disc of radius r about (cx, cy) inside [x0, x1] x [y0, y1],
    by adaptive quadrature of the disc's vertical chord clipped to the cell."""
    a, b = max(x0, cx - r), min(x1, cx + r)
    if b <= a:
        return 0.0

    def chord(x):
        s = math.sqrt(max(r * r - (x - cx) ** 2, 0.0))
        return max(0.0, min(y1, cy + s) - max(y0, cy - s))

    kinks = []
    for yb in (y0, y1):  # where the circle crosses the cell's horizontal edges
        d = yb - cy
        if abs(d) < r:
            for sgn in (-1, 1):
                x = cx + sgn * math.sqrt(r * r - d * d)
                if a < x < b:
                    kinks.append(x)
    val, _ = integrate.quad(chord, a, b, points=sorted(kinks) or None, epsabs=1e-17, epsrel=1e-13,
                            limit=200)
    return val


def probe_cells(p, centres=PROBE_CENTRES, r=PROBE_RADIUS, n_windows=N_WINDOWS):
    """Cells of every probe ball with weight = (area of the cell in the ball) / (pi r^2),
    as the dict ``oracle.solve(..., probes=...)`` takes."""
    ci, cj, pr, wt = [], [], [], []
    for q, (cx, cy) in enumerate(centres):
        for j in range(p.ny):
            y0, y1 = p.y0 + j * p.h, p.y0 + (j + 1) * p.h
            if y1 <= cy - r or y0 >= cy + r:
                continue
            for i in range(p.nx):
                x0, x1 = p.x0 + i * p.h, p.x0 + (i + 1) * p.h
                if x1 <= cx - r or x0 >= cx + r:
                    continue
                area = disc_cell_area(cx, cy, r, x0, x1, y0, y1)
                if area > 1e-9 * p.h * p.h:  # not a rounding sliver of a cell the disc only touches
                    ci.append(i)
                    cj.append(j)
                    pr.append(q)
                    wt.append(area / (math.pi * r * r))
    return dict(n_probes=len(centres), n_windows=n_windows, cell_i=np.array(ci), cell_j=np.array(cj),
                probe=np.array(pr), weight=np.array(wt))
