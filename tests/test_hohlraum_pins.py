"""Pins of the Hohlraum workload (Sec. 3.2.1) and of the oracle on it.

The layout is checked against the areas of the paper's set definitions and
its mirror symmetry in both axes; the oracle's solution against that
symmetry, the particle balance, and the inflow through the two irradiated
sides, whose trace is the prescribed value whatever the interior does.
"""

import json
import os

import numpy as np
import pytest

from paper_2505_17284_amd import inputs as I
from tests.conftest import qdict

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Areas of the sets of Sec. 3.2.1 (black, red, green, blue) from their
# defining intervals; white is the rest of the 1.3 x 1.3 square.
AREA = {
    "K": 2 * 1.3 * 0.05,
    "R": 2 * 0.05 * 0.8,
    "G": 2 * 0.05 * 0.7 + 2 * 0.40 * 0.05,
    "B": 0.30 * 0.70,
}
AREA["W"] = 1.3 * 1.3 - sum(AREA.values())


@pytest.mark.parametrize("n", [26, 52, 260])
def test_layout_areas_aligned_grids(n):
    r = I.hohlraum_region_map(n)
    h2 = (1.3 / n) ** 2
    for k, name in enumerate(I.HOHLRAUM_REGIONS):
        assert int((r == k).sum()) * h2 == pytest.approx(AREA[name], rel=1e-12, abs=1e-12), name


@pytest.mark.parametrize("n", [100, 333])
def test_layout_areas_unaligned_grids_within_a_cell_layer(n):
    r = I.hohlraum_region_map(n)
    h = 1.3 / n
    perimeter = {"K": 2 * (2 * 1.3 + 2 * 0.05), "R": 2 * (2 * 0.05 + 2 * 0.8),
                 "G": 2 * (2 * 0.4 + 2 * 0.8), "B": 2 * (0.3 + 0.7)}
    for k, name in enumerate(I.HOHLRAUM_REGIONS[1:], start=1):
        assert abs(int((r == k).sum()) * h * h - AREA[name]) <= perimeter[name] * h, name


def test_layout_mirror_symmetric_and_green_ring_closed():
    r = I.hohlraum_region_map(52)
    assert np.array_equal(r, r[:, ::-1]) and np.array_equal(r, r[::-1, :])
    # the capsule interior is enclosed by green: every blue cell's neighbours are blue or green
    b = r == 1
    for dj, di in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        nb = np.roll(np.roll(r, dj, 0), di, 1)
        assert np.all(np.isin(nb[b], (1, 3)))


@pytest.mark.parametrize("order", [1, 2])
def test_oracle_mirror_symmetry_both_axes(orc, order):
    """The layout, the inflow and the quadrature are symmetric under x -> -x
    and y -> -y, so psi_k(i, j) = psi_{rx(k)}(n-1-i, j) = psi_{ry(k)}(i, n-1-j).
    First order: to rounding. Second order: the mirrored cell sums phi over its
    ordinates in another order, and where the minmod limiter switches branch
    such last-bit differences are amplified (they start at 1e-14, saturate
    near 1e-6 of the peak over the whole run on grids of 104-156 cells and
    do not grow further); an index or sign error breaks the symmetry at O(1)."""
    p = I.hohlraum(104, 32, order=order, t_end=0.6)  # stable and positive from about 104 cells (sigma_t = 100)
    psi = orc.solve(p)["psi"]
    qd = p.quad
    atol = 1e-15 if order == 1 else 1e-5 * float(np.abs(psi).max())
    rtol = 1e-12 if order == 1 else 0.0
    np.testing.assert_allclose(psi, psi[qd.mirror_x][:, :, ::-1], rtol=rtol, atol=atol)
    np.testing.assert_allclose(psi, psi[qd.mirror_y][:, ::-1, :], rtol=rtol, atol=atol)


def test_oracle_balance_and_prescribed_inflow(orc):
    """mass(T) = int (inflow - outflow - absorption) dt exactly (no source, no
    initial particles), and the instantaneous inflow through the domain
    boundary is 2 x 1.3 x sum_{xi > 0} w xi at every time: the entering trace
    on both irradiated sides is the prescribed 1, on the others 0."""
    p = I.hohlraum(104, 32, order=2, t_end=0.8)
    r = orc.solve(p)
    q, qi = qdict(r["names"], r["qoi"]), qdict(r["names"], r["qoi_int"])
    qd = p.quad
    rate = 2 * 1.3 * float(np.sum(qd.w[qd.xi > 0] * qd.xi[qd.xi > 0]))
    assert q["in:domain"] == pytest.approx(rate, rel=1e-13)
    assert qi["in:domain"] == pytest.approx(rate * p.t_end, rel=1e-12)
    assert qi["source"] == 0.0
    gain = qi["in:domain"] - qi["out:domain"] - sum(qi[f"abs:{t}"] for t in p.tally_names)
    assert abs(q["mass"] - gain) <= 1e-12 * qi["in:domain"]
    assert qi["abs:W"] == 0.0  # sigma_a = 0 in the white region


def test_oracle_reference_run_plausible_against_the_paper():
    """The stored oracle run (260^2 cells, 256 ordinates, minmod, Heun, CFL
    0.5) against the paper's Hohlraum table (unstructured mesh at h <= 1e-3,
    tessellation quadrature, Venkatakrishnan limiter): a different
    discretisation, so only a loose band, but the same problem."""
    path = os.path.join(GOLDEN, "oracle_hohlraum260_M256_heun2.json")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    with open(path) as f:
        g = json.load(f)
    with open(os.path.join(GOLDEN, "paper_hohlraum_table.json")) as f:
        tab = json.load(f)
    pairs = [("abs:GB", "QoI-2 G+B"), ("abs:R", "QoI-2 R"), ("abs:K", "QoI-2 K")]
    for ours, theirs in pairs:
        assert g["qoi_int"][ours] == pytest.approx(tab[theirs]["mean"], rel=0.15), ours
    assert g["qoi"]["mass"] == pytest.approx(tab["QoI-7"]["mean"], rel=0.15)
    # QoI-3 and QoI-4 (green blocks, oracle/hohlraum_qoi.py on the oracle's
    # fluence) land as close as QoI-2 does. QoI-5/6 are means of the same
    # field along the blocks' centre line, so by their definitions A_L is of
    # the order of A_G; the table prints them two orders of magnitude lower,
    # which no reading of the definitions reproduces: compared by order only.
    band = g["green_band"]
    assert band["A_G"] == pytest.approx(tab["QoI-3"]["mean"], rel=0.15)
    assert band["V_G"] == pytest.approx(tab["QoI-4"]["mean"], rel=0.15)
    assert 0.25 * band["A_G"] < band["A_L"] < band["A_G"]
    assert band["length"] == pytest.approx(2.2, rel=1e-12)


def test_oracle_probe_windows_show_the_papers_symmetry():
    """QoI-1 of the stored run: the paper observes that the two probes left
    and right of the capsule share phi and J_y and have opposite J_x, the two
    above and below share phi and J_x and have opposite J_y, and each pair's
    cross current vanishes (R23 bounds the mirror defect at second order)."""
    with open(os.path.join(GOLDEN, "oracle_hohlraum260_M256_heun2.json")) as f:
        g = json.load(f)
    if "probes" not in g:
        pytest.skip("golden has no probe values")
    a = np.array(g["probes"])  # [window][probe][phi, J_x, J_y]
    tol = 1e-5 * np.abs(a[:, :, 0]).max()
    for lo, hi, axis in ((0, 1, 1), (2, 3, 2)):
        other = 3 - axis
        assert np.abs(a[:, lo, 0] - a[:, hi, 0]).max() <= tol
        assert np.abs(a[:, lo, axis] + a[:, hi, axis]).max() <= tol
        assert np.abs(a[:, lo, other]).max() <= tol and np.abs(a[:, hi, other]).max() <= tol
    assert a[-1, 0, 0] > 0.5 and a[-1, 0, 1] > 0  # particles reach the probe and stream inwards
