"""Seeded problem statements for the S_N transport step.

This module only *states* problems: geometry masks on a uniform Cartesian
grid, per-region cross-sections and sources, boundary data, an angular
quadrature, the QoI regions and rectangles, and seeded random draws. It holds
none of the method's arithmetic (no time-step count, no fluxes, no QoIs): the
native library and the FP64 oracle each derive those from the statement on
their own.

Paper references (arXiv 2505.17284):
  * S_N system on the upper hemisphere, weights summing to 2*pi: Sec. 4.1,
    eq. ``eq_sn_2d``.
  * Lattice benchmark geometry, materials, T = 3.2: Sec. 3.1.1 and the
    material table of the lattice figure; QoI regions S_l: Sec. 3.1.2.
  * Lattice design parameters DP-2 (per-block cross-sections): Sec. 3.1.3.
  * Tensorised Gauss-Legendre quadrature, named as the alternative to the
    tessellation rule: Sec. 5.1.1.

Readings where the paper does not fix the statement (product quadrature
layout, the walled cavity, the random draw order) are listed in the design doc.
"""

from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

# Boundary kinds, in side order W, E, S, N.
BC_VACUUM = 0
BC_INFLOW = 1
BC_REFLECT = 2
SIDE_W, SIDE_E, SIDE_S, SIDE_N = 0, 1, 2, 3

EULER = 0
HEUN = 1

# Hard limits shared by the C ABI (include/snrt.h) and the oracle.
MAX_TALLIES = 8
MAX_RECTS = 4
MAX_REGIONS = 256

# Ordinate counts used by the benchmark configurations -> (polar, azimuthal).
M_SPLIT = {32: (4, 8), 64: (4, 16), 128: (8, 16), 256: (8, 32), 512: (8, 64)}


@dataclass
class Quadrature:
    """Ordinates Omega_k = (xi_k, eta_k, mu_k) on the upper hemisphere."""

    mu: np.ndarray
    xi: np.ndarray
    eta: np.ndarray
    w: np.ndarray
    mirror_x: np.ndarray  # index of the ordinate with xi -> -xi
    mirror_y: np.ndarray  # index of the ordinate with eta -> -eta
    n_polar: int
    n_azim: int

    @property
    def M(self) -> int:
        return int(self.w.shape[0])


@dataclass
class Problem:
    """A complete statement of one S_N solve on a uniform square grid.

    ``region[j, i]`` is the material id of cell (i, j), i along x; cell (i, j)
    covers [x0 + i h, x0 + (i+1) h] x [y0 + j h, y0 + (j+1) h].
    ``rects[q] = (i0, j0, i1, j1)`` is the half-open cell range whose boundary
    carries the outflow/inflow QoI number q.
    """

    name: str
    nx: int
    ny: int
    h: float
    x0: float
    y0: float
    quad: Quadrature
    region: np.ndarray
    sigma_a: np.ndarray
    sigma_s: np.ndarray
    q: np.ndarray
    tally: np.ndarray
    tally_names: list
    bc: tuple
    inflow: tuple
    order: int
    stepper: int
    cfl: float
    t_end: float
    rects: np.ndarray
    rect_names: list
    psi_dtype: str = "f32"
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return self.quad.M

    @property
    def n_regions(self) -> int:
        return int(self.sigma_a.shape[0])

    @property
    def n_tallies(self) -> int:
        return len(self.tally_names)

    @property
    def n_rects(self) -> int:
        return int(self.rects.shape[0])

    @property
    def cell_ordinates(self) -> int:
        return int(self.nx) * int(self.ny) * self.M

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Quadrature (Sec. 5.1.1 names tensorised Gauss-Legendre as the alternative to
# the tessellation rule; weights normalised to 2*pi over S^2_+ per Sec. 4.1).
# --------------------------------------------------------------------------

def product_quadrature(n_polar: int, n_azim: int, half_range: bool = False) -> Quadrature:
    """Gauss-Legendre in mu times uniform midpoint azimuths, ordered k = p*n_azim + q.

    Polar nodes are the positive half of the 2*n_polar-point Gauss-Legendre
    rule on [-1, 1] (their weights sum to 1); with ``half_range`` they are the
    n_polar-point rule mapped to [0, 1]. Azimuths are (q + 1/2) 2 pi / n_azim
    and every weight is w_p * 2 pi / n_azim, so the weights sum to 2 pi.

    Only the first octant is evaluated with cos/sin; the rest of the circle is
    filled by swapping (xi, eta) and flipping signs, so mirror partners are
    exact in floating point: xi[mirror_x[k]] == -xi[k] bit for bit, and the
    set is closed under the transpose xi <-> eta.
    """
    if n_polar < 1 or n_azim < 8 or n_azim % 8 != 0:
        raise ValueError("need n_polar >= 1 and n_azim a positive multiple of 8")
    if half_range:
        x, wp = np.polynomial.legendre.leggauss(n_polar)
        mu = 0.5 * (x + 1.0)
        wp = 0.5 * wp
    else:
        x, wp = np.polynomial.legendre.leggauss(2 * n_polar)
        mu = x[n_polar:].copy()
        wp = wp[n_polar:].copy()
    nq = n_azim
    c = np.empty(nq)
    s = np.empty(nq)
    oct_n = nq // 8
    for q in range(oct_n):
        ang = (q + 0.5) * 2.0 * np.pi / nq
        c[q], s[q] = np.cos(ang), np.sin(ang)
    for q in range(oct_n):  # second half of quadrant 1 by the transpose
        c[nq // 4 - 1 - q], s[nq // 4 - 1 - q] = s[q], c[q]
    for q in range(nq // 4):  # quadrant 2: xi -> -xi
        c[nq // 2 - 1 - q], s[nq // 2 - 1 - q] = -c[q], s[q]
    for q in range(nq // 2):  # quadrants 3, 4: eta -> -eta
        c[nq - 1 - q], s[nq - 1 - q] = c[q], -s[q]
    M = n_polar * nq
    mu_k = np.repeat(mu, nq)
    sin_t = np.sqrt(1.0 - mu * mu)
    xi = (sin_t[:, None] * c[None, :]).reshape(M)
    eta = (sin_t[:, None] * s[None, :]).reshape(M)
    w = (wp[:, None] * np.full(nq, 2.0 * np.pi / nq)[None, :]).reshape(M)
    qs = np.arange(nq)
    qx = (nq // 2 - 1 - qs) % nq
    qy = nq - 1 - qs
    p = np.arange(n_polar)
    mirror_x = (p[:, None] * nq + qx[None, :]).reshape(M).astype(np.int32)
    mirror_y = (p[:, None] * nq + qy[None, :]).reshape(M).astype(np.int32)
    return Quadrature(mu=mu_k, xi=xi, eta=eta, w=w, mirror_x=mirror_x,
                      mirror_y=mirror_y, n_polar=n_polar, n_azim=n_azim)


def tessellation_quadrature(N: int) -> Quadrature:
    """The tessellation rule of Sec. 5.1.1: M = 4 N^2 ordinates on S^2_+.

    Each face of the octahedron with vertices on the unit sphere is cut into
    N^2 triangles by the lines parallel to its edges through the points that
    divide the edges into N parts. An ordinate is the centroid of one such
    planar triangle pushed out to the unit sphere; its weight is the area of
    the spherical triangle spanned by the pushed-out vertices (its spherical
    excess E, from tan(E/2) = |a . (b x c)| / (1 + a.b + b.c + c.a)). The
    weights tile the hemisphere, so they sum to 2 pi.

    The face in the first octant is computed; the other three faces of the
    upper hemisphere are its images under xi -> -xi and eta -> -eta, so mirror
    partners are exact. Order: k = f N^2 + t, faces f = (+,+), (-,+), (-,-),
    (+,-) in (xi, eta), triangles t of the first face as generated.
    """
    if N < 1:
        raise ValueError("need N >= 1")

    def node(i, j):  # barycentric grid point of the face x + y + z = 1
        return np.array([i / N, j / N, (N - i - j) / N])

    tris = []
    for i in range(N):
        for j in range(N - i):
            tris.append((node(i, j), node(i + 1, j), node(i, j + 1)))
            if i + j <= N - 2:
                tris.append((node(i + 1, j), node(i + 1, j + 1), node(i, j + 1)))
    n1 = len(tris)
    pts = np.empty((n1, 3))
    wts = np.empty(n1)
    for t, (a, b, c) in enumerate(tris):
        g = (a + b + c) / 3.0
        pts[t] = g / np.linalg.norm(g)
        ua, ub, uc = (v / np.linalg.norm(v) for v in (a, b, c))
        num = abs(np.dot(ua, np.cross(ub, uc)))
        den = 1.0 + np.dot(ua, ub) + np.dot(ub, uc) + np.dot(uc, ua)
        wts[t] = 2.0 * np.arctan2(num, den)
    sx = np.array([1.0, -1.0, -1.0, 1.0])
    sy = np.array([1.0, 1.0, -1.0, -1.0])
    xi = (sx[:, None] * pts[None, :, 0]).reshape(-1)
    eta = (sy[:, None] * pts[None, :, 1]).reshape(-1)
    mu = np.tile(pts[:, 2], 4)
    w = np.tile(wts, 4)
    t = np.arange(n1)
    fx = np.array([1, 0, 3, 2])  # face of the xi-mirror
    fy = np.array([3, 2, 1, 0])  # face of the eta-mirror
    mirror_x = (fx[:, None] * n1 + t[None, :]).reshape(-1).astype(np.int32)
    mirror_y = (fy[:, None] * n1 + t[None, :]).reshape(-1).astype(np.int32)
    return Quadrature(mu=mu, xi=xi, eta=eta, w=w, mirror_x=mirror_x, mirror_y=mirror_y,
                      n_polar=N, n_azim=0)


def quadrature_for(M: int) -> Quadrature:
    if M not in M_SPLIT:
        raise ValueError(f"no product split registered for M={M}")
    return product_quadrature(*M_SPLIT[M])


# --------------------------------------------------------------------------
# Lattice benchmark (Sec. 3.1.1), shifted from [-3.5, 3.5]^2 to [0, 7]^2.
# Block C_{i,j} (1-based, i along x) covers [i-1, i] x [j-1, j].
# --------------------------------------------------------------------------

LATTICE_ABSORBER_BLOCKS = [(2, 2), (4, 2), (6, 2), (3, 3), (5, 3), (2, 4),
                           (6, 4), (3, 5), (5, 5), (2, 6), (6, 6)]
LATTICE_SOURCE_BLOCK = (4, 4)
LATTICE_TALLIES = ["W", "B", "R"]  # white (scatterer), blue (absorber), red (source)


def lattice_block_kind(d4: bool = False) -> np.ndarray:
    """kind[J, I] for 0-based block (I, J): 0 = W, 1 = B, 2 = R.

    ``d4`` adds C_{4,6} to B, which makes the layout symmetric under the full
    square group (a test-only variant; the paper's lattice mirrors in x only).
    """
    kind = np.zeros((7, 7), dtype=np.int32)
    blocks = list(LATTICE_ABSORBER_BLOCKS) + ([(4, 6)] if d4 else [])
    for (i, j) in blocks:
        kind[j - 1, i - 1] = 1
    i, j = LATTICE_SOURCE_BLOCK
    kind[j - 1, i - 1] = 2
    return kind


def _lattice_cell_blocks(n: int) -> np.ndarray:
    """0-based block index of every cell centre along one axis (exact integers)."""
    i = np.arange(n, dtype=np.int64)
    # centre (i + 1/2) * 7 / n lies in block floor((2i + 1) * 7 / (2n)); never a tie
    return ((2 * i + 1) * 7) // (2 * n)


def _lattice_rects(n: int):
    rects = [(0, 0, n, n)]
    names = ["domain"]
    snapped = {}
    for ell in (1.5, 2.5):
        lo = int(np.floor((3.5 - ell) * n / 7.0 + 0.5))
        hi = n - lo
        rects.append((lo, lo, hi, hi))
        names.append(f"S_{ell}")
        snapped[ell] = (hi - lo) * 7.0 / (2 * n)
    return np.array(rects, dtype=np.int32), names, snapped


def lattice(n: int = 70, M: int = 32, order: int = 1, stepper: int = EULER,
            cfl: float = 0.5, t_end: float = 3.2, per_block=None, d4: bool = False,
            bc=(BC_VACUUM,) * 4, psi_dtype: str = "f32", quad: Quadrature | None = None,
            name: str | None = None) -> Problem:
    """The lattice benchmark on an n x n grid over [0, 7]^2.

    Nominal materials: W sigma_s = 1; B sigma_a = 10; R sigma_s = 1, Q = 1
    (lattice material table). ``per_block`` = (sigma_a[49], sigma_s[49], q[49])
    gives every block its own region (DP-2); tallies stay W/B/R.
    """
    quad = quad if quad is not None else quadrature_for(M)
    kind = lattice_block_kind(d4)
    bi = _lattice_cell_blocks(n)
    block_id = bi[None, :] + 7 * bi[:, None]  # [ny, nx] -> J*7 + I
    kind_flat = kind.reshape(49)
    if per_block is None:
        region = kind_flat[block_id].astype(np.uint8)
        sigma_a = np.array([0.0, 10.0, 0.0])
        sigma_s = np.array([1.0, 0.0, 1.0])
        q = np.array([0.0, 0.0, 1.0])
        tally = np.array([0, 1, 2], dtype=np.uint8)
    else:
        sa, ss, qq = (np.asarray(a, dtype=np.float64).reshape(49) for a in per_block)
        region = block_id.astype(np.uint8)
        sigma_a, sigma_s, q = sa.copy(), ss.copy(), qq.copy()
        tally = kind_flat.astype(np.uint8)
    rects, rect_names, snapped = _lattice_rects(n)
    return Problem(
        name=name or f"lattice_n{n}_M{quad.M}",
        nx=n, ny=n, h=7.0 / n, x0=0.0, y0=0.0, quad=quad,
        region=np.ascontiguousarray(region), sigma_a=sigma_a, sigma_s=sigma_s, q=q,
        tally=tally, tally_names=list(LATTICE_TALLIES), bc=tuple(bc),
        inflow=(0.0, 0.0, 0.0, 0.0), order=order, stepper=stepper, cfl=cfl,
        t_end=t_end, rects=rects, rect_names=rect_names, psi_dtype=psi_dtype,
        meta={"kind": "lattice", "snapped_ell": snapped, "d4": d4},
    )


# --------------------------------------------------------------------------
# Walled cavity: domain [-0.65, 0.65]^2, absorbing walls 0.05 thick on all
# sides, an inner [-0.4, 0.4]^2 absorber, void elsewhere, isotropic inflow
# psi = 1 on the west side. Lengths are integers in units of 0.05 (26 across).
# --------------------------------------------------------------------------

CAVITY_TALLIES = ["void", "wall", "block"]


def _cavity_centres_scaled(n: int) -> np.ndarray:
    """n * (cell centre in units of 0.05), exact: -13 n + 13 (2 i + 1)."""
    i = np.arange(n, dtype=np.int64)
    return -13 * n + 13 * (2 * i + 1)


def cavity(n: int = 1300, M: int = 512, order: int = 2, stepper: int = HEUN,
           cfl: float = 0.5, t_end: float = 2.6, open_left: bool = False,
           psi_dtype: str = "f32", quad: Quadrature | None = None,
           name: str | None = None) -> Problem:
    quad = quad if quad is not None else quadrature_for(M)
    c = _cavity_centres_scaled(n)

    def inside(lo, hi):  # half-open [lo, hi) in units of 0.05
        return (c >= lo * n) & (c < hi * n)

    inner_x, inner_y = inside(-12, 12), inside(-12, 12)
    blk_x, blk_y = inside(-8, 8), inside(-8, 8)
    if open_left:
        wall_x = c >= 12 * n
        wall = wall_x[None, :] | (~inner_y)[:, None]
    else:
        wall = (~inner_x)[None, :] | (~inner_y)[:, None]
    block = blk_x[None, :] & blk_y[:, None]
    region = np.zeros((n, n), dtype=np.uint8)
    region[wall] = 1
    region[block] = 2
    lo = int(np.floor(5 * n / 26.0 + 0.5))  # x = -0.4 -> (0.25 / 1.3) n
    rects = np.array([(0, 0, n, n), (lo, lo, n - lo, n - lo)], dtype=np.int32)
    return Problem(
        name=name or f"cavity_n{n}_M{quad.M}",
        nx=n, ny=n, h=1.3 / n, x0=-0.65, y0=-0.65, quad=quad, region=region,
        sigma_a=np.array([0.0, 100.0, 100.0]), sigma_s=np.array([0.0, 0.1, 0.0]),
        q=np.zeros(3), tally=np.array([0, 1, 2], dtype=np.uint8),
        tally_names=list(CAVITY_TALLIES),
        bc=(BC_INFLOW, BC_VACUUM, BC_VACUUM, BC_VACUUM), inflow=(1.0, 0.0, 0.0, 0.0),
        order=order, stepper=stepper, cfl=cfl, t_end=t_end, rects=rects,
        rect_names=["domain", "block"], psi_dtype=psi_dtype,
        meta={"kind": "cavity", "open_left": open_left},
    )


# --------------------------------------------------------------------------
# Hohlraum benchmark (Sec. 3.2.1) on D = [-0.65, 0.65]^2. Every edge of the
# layout lies on a multiple of 0.05, so for n a multiple of 26 the material
# interfaces are cell faces. Blocks in units of 0.05 (open sets; cells are
# assigned by their centres, half-open [lo, hi)):
#   K (black)  (-13, 13) x (-13, -12) and (-13, 13) x (12, 13)
#   R (red)    (-13, -12) x (-8, 8)   and (12, 13) x (-8, 8)
#   G (green)  (-4, -3) x (-7, 7), (3, 4) x (-7, 7), (-4, 4) x (-8, -7), (-4, 4) x (7, 8)
#   B (blue, capsule interior; not defined in the text, read off G) (-3, 3) x (-7, 7)
#   W (white)  the rest
# Materials from the table of the Hohlraum figure (sigma_a, sigma_s):
# W (0, 0.1), B (100, 0), R (5, 95), G (10, 90), K (50, 50). No source, no
# initial particles, isotropic inflow 1 through x = -0.65 (xi > 0) and
# x = 0.65 (xi < 0), vacuum elsewhere, T = 2.6.
# --------------------------------------------------------------------------

HOHLRAUM_REGIONS = ["W", "B", "R", "G", "K"]
HOHLRAUM_SIGMA_A = [0.0, 100.0, 5.0, 10.0, 50.0]
HOHLRAUM_SIGMA_S = [0.1, 0.0, 95.0, 90.0, 50.0]
HOHLRAUM_TALLIES = ["GB", "R", "K", "W"]  # absorption QoI-2 over G u B, R, K; W closes the balance
HOHLRAUM_REGION_TALLY = [3, 0, 1, 0, 2]


def hohlraum_region_map(n: int) -> np.ndarray:
    """region[j, i] of the Hohlraum layout on an n x n grid (ids of HOHLRAUM_REGIONS)."""
    c = _cavity_centres_scaled(n)  # n * cell centre in units of 0.05

    def inside(lo, hi):
        return (c >= lo * n) & (c < hi * n)

    def box(x_lo, x_hi, y_lo, y_hi):
        return inside(y_lo, y_hi)[:, None] & inside(x_lo, x_hi)[None, :]

    region = np.zeros((n, n), dtype=np.uint8)
    region[box(-13, 13, -13, -12) | box(-13, 13, 12, 13)] = 4
    region[box(-13, -12, -8, 8) | box(12, 13, -8, 8)] = 2
    region[box(-4, -3, -7, 7) | box(3, 4, -7, 7) | box(-4, 4, -8, -7) | box(-4, 4, 7, 8)] = 3
    region[box(-3, 3, -7, 7)] = 1
    return region


def hohlraum(n: int = 260, M: int = 128, order: int = 2, stepper: int = HEUN, cfl: float = 0.5,
             t_end: float = 2.6, psi_dtype: str = "f32", quad: Quadrature | None = None,
             name: str | None = None) -> Problem:
    quad = quad if quad is not None else quadrature_for(M)
    return Problem(
        name=name or f"hohlraum_n{n}_M{quad.M}",
        nx=n, ny=n, h=1.3 / n, x0=-0.65, y0=-0.65, quad=quad, region=hohlraum_region_map(n),
        sigma_a=np.array(HOHLRAUM_SIGMA_A), sigma_s=np.array(HOHLRAUM_SIGMA_S), q=np.zeros(5),
        tally=np.array(HOHLRAUM_REGION_TALLY, dtype=np.uint8), tally_names=list(HOHLRAUM_TALLIES),
        bc=(BC_INFLOW, BC_INFLOW, BC_VACUUM, BC_VACUUM), inflow=(1.0, 1.0, 0.0, 0.0),
        order=order, stepper=stepper, cfl=cfl, t_end=t_end, rects=np.array([(0, 0, n, n)], dtype=np.int32),
        rect_names=["domain"], psi_dtype=psi_dtype, meta={"kind": "hohlraum"},
    )


# --------------------------------------------------------------------------
# Test problems with closed-form behaviour.
# --------------------------------------------------------------------------

def homogeneous(nx: int = 6, ny: int = 5, M: int = 32, sigma_a: float = 0.7,
                sigma_s: float = 0.4, q: float = 1.3, order: int = 1,
                stepper: int = EULER, cfl: float = 0.5, t_end: float = 1.0,
                h: float = 0.1) -> Problem:
    """Uniform medium closed by reflective walls: an infinite medium."""
    quad = quadrature_for(M)
    return Problem(
        name="homogeneous", nx=nx, ny=ny, h=h, x0=0.0, y0=0.0, quad=quad,
        region=np.zeros((ny, nx), dtype=np.uint8), sigma_a=np.array([sigma_a]),
        sigma_s=np.array([sigma_s]), q=np.array([q]), tally=np.array([0], np.uint8),
        tally_names=["all"], bc=(BC_REFLECT,) * 4, inflow=(0.0,) * 4, order=order,
        stepper=stepper, cfl=cfl, t_end=t_end,
        rects=np.array([(0, 0, nx, ny)], dtype=np.int32), rect_names=["domain"],
    )


def beam(nx: int = 24, ny: int = 3, M: int = 32, sigma: float = 2.0, g: float = 1.0,
         h: float = 0.05, order: int = 1, stepper: int = EULER, cfl: float = 0.5,
         t_end: float = 1.0) -> Problem:
    """Pure absorber, y-uniform: inflow g on W, vacuum E, reflective S and N."""
    quad = quadrature_for(M)
    return Problem(
        name="beam", nx=nx, ny=ny, h=h, x0=0.0, y0=0.0, quad=quad,
        region=np.zeros((ny, nx), dtype=np.uint8), sigma_a=np.array([sigma]),
        sigma_s=np.array([0.0]), q=np.array([0.0]), tally=np.array([0], np.uint8),
        tally_names=["all"], bc=(BC_INFLOW, BC_VACUUM, BC_REFLECT, BC_REFLECT),
        inflow=(g, 0.0, 0.0, 0.0), order=order, stepper=stepper, cfl=cfl, t_end=t_end,
        rects=np.array([(0, 0, nx, ny)], dtype=np.int32), rect_names=["domain"],
    )


def random_materials(nx: int, ny: int, n_regions: int, seed: int, M: int = 32,
                     order: int = 2, stepper: int = HEUN, bc=(BC_VACUUM,) * 4,
                     inflow=(0.0,) * 4, cfl: float = 0.5, t_end: float = 0.5,
                     h: float = 0.05, rects=None, n_tallies: int = 3,
                     psi_dtype: str = "f32") -> Problem:
    """Random region map and cross-sections: exercises every code path."""
    rng = np.random.Generator(np.random.PCG64(seed))
    quad = quadrature_for(M)
    region = rng.integers(0, n_regions, size=(ny, nx)).astype(np.uint8)
    sigma_a = rng.uniform(0.0, 5.0, n_regions)
    sigma_s = rng.uniform(0.0, 3.0, n_regions)
    q = rng.uniform(0.0, 1.0, n_regions)
    tally = (np.arange(n_regions) % n_tallies).astype(np.uint8)
    if rects is None:
        rects = [(0, 0, nx, ny)]
        if nx >= 4 and ny >= 4:
            rects.append((1, 1, nx - 1, ny - 1))
        if nx >= 6 and ny >= 5:
            rects.append((2, 1, nx - 3, ny - 2))
    rects = np.array(rects, dtype=np.int32)
    return Problem(
        name=f"random_{nx}x{ny}_s{seed}", nx=nx, ny=ny, h=h, x0=0.0, y0=0.0,
        quad=quad, region=region, sigma_a=sigma_a, sigma_s=sigma_s, q=q,
        tally=tally, tally_names=[f"t{t}" for t in range(n_tallies)], bc=tuple(bc),
        inflow=tuple(inflow), order=order, stepper=stepper, cfl=cfl, t_end=t_end,
        rects=rects, rect_names=[f"r{r}" for r in range(len(rects))],
        psi_dtype=psi_dtype,
    )


def random_state(p: Problem, seed: int, kind: str = "uniform") -> np.ndarray:
    """A seeded angular flux [M, ny, nx] whose values are exact in FP32 (and,
    for ``psi_dtype == 'bf16'``, exact in BF16)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (p.M, p.ny, p.nx)
    if kind == "uniform":
        a = rng.uniform(0.0, 1.0, shape)
    elif kind == "smooth":
        yy, xx = np.meshgrid(np.arange(p.ny), np.arange(p.nx), indexing="ij")
        base = 1.0 + 0.5 * np.sin(0.4 * xx + 0.1) * np.cos(0.3 * yy)
        a = base[None] * rng.uniform(0.5, 1.5, (p.M, 1, 1)) + 0.05 * rng.uniform(-1, 1, shape)
    else:
        raise ValueError(kind)
    a = a.astype(np.float32)
    if p.psi_dtype == "bf16":
        bits = a.view(np.uint32) & np.uint32(0xFFFF0000)
        a = bits.view(np.float32)
    return a.astype(np.float64)


# --------------------------------------------------------------------------
# Benchmark configurations.
# --------------------------------------------------------------------------

def config(i: int) -> Problem:
    """The five benchmark configurations (cfg 4 and 5 are generators)."""
    if i == 1:  # 70^2, 32 ordinates, first order, forward Euler
        return lattice(70, 32, order=1, stepper=EULER, name="lattice70_M32_euler1")
    if i == 2:  # 700^2, 256 ordinates, minmod, Heun
        return lattice(700, 256, order=2, stepper=HEUN, name="lattice700_M256_heun2")
    if i == 3:  # walled cavity 1300^2, 512 ordinates, minmod, Heun
        return cavity(1300, 512, name="cavity1300_M512_heun2")
    raise ValueError("configs 4 and 5 are generated by uq_instance / serving_requests")


def _draw_dp2(rng):
    """DP-2 draw: sigma_a ~ U[5, 15] for the 11 absorber blocks in (j, i)
    row-major order, sigma_s ~ U[0.5, 1.5] for the 38 other blocks, then
    q ~ U[0.5, 1.5] for the source block."""
    kind = lattice_block_kind().reshape(49)
    sa = np.zeros(49)
    ss = np.zeros(49)
    qq = np.zeros(49)
    b_idx = [b for b in range(49) if kind[b] == 1]
    o_idx = [b for b in range(49) if kind[b] != 1]
    sa[b_idx] = rng.uniform(5.0, 15.0, len(b_idx))
    ss[o_idx] = rng.uniform(0.5, 1.5, len(o_idx))
    r = [b for b in range(49) if kind[b] == 2][0]
    qq[r] = rng.uniform(0.5, 1.5)
    return sa, ss, qq


def uq_instance(seed: int, psi_dtype: str = "f32") -> Problem:
    """One DP-2 lattice draw: n, then M, then the cross-sections (``_draw_dp2``)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.choice([140, 280, 420, 560]))
    M = int(rng.choice([64, 128, 256]))
    per_block = _draw_dp2(rng)
    return lattice(n, M, order=2, stepper=HEUN, per_block=per_block,
                   psi_dtype=psi_dtype, name=f"uq_s{seed}_n{n}_M{M}")


def serving_requests(n_requests: int, rate: float, seed: int = 0,
                     dtypes=("f32",), n_range=(100, 1000)):
    """Poisson arrivals of mixed lattice / cavity requests.

    Returns a list of (arrival_time_s, Problem). Lattice requests draw
    cross-sections like ``uq_instance``; cavity requests use nominal values.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        kind = "lattice" if rng.uniform() < 0.5 else "cavity"
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        M = int(rng.choice([32, 64, 128, 256, 512]))
        dt = dtypes[int(rng.integers(0, len(dtypes)))]
        if kind == "lattice":
            p = lattice(n, M, order=2, stepper=HEUN, per_block=_draw_dp2(rng),
                        psi_dtype=dt, name=f"req{r}_lattice_n{n}_M{M}")
        else:
            p = cavity(n, M, psi_dtype=dt, name=f"req{r}_cavity_n{n}_M{M}")
        out.append((t, p))
    return out
