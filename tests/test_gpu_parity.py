"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every input comes from the seeded generators; every expected value from the
oracle (or from a committed golden written by a script that calls only the
oracle). Cases span several tiles (128 columns per wave, 4 waves of 2 rows
per workgroup) with ragged tails in x and y, every boundary kind, both orders
and both steppers, and the degenerate grids.
"""

import json
import os

import numpy as np
import pytest

from paper_2505_17284_amd import inputs as I
from tests.parity import compare_field, compare_qoi

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def sv():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17284_amd import solver

    return solver


def _orc_dicts(r):
    return dict(zip(r["names"], r["qoi"])), dict(zip(r["names"], r["qoi_int"]))


def _run_both(sv, orc, p, steps, psi0=None, **kw):
    print(f"[case] {p.name} n=({p.nx},{p.ny}) M={p.M} order={p.order} stepper={p.stepper} "
          f"bc={p.bc} dtype={p.psi_dtype} steps={steps} kw={kw}", flush=True)
    g = sv.solve(p, steps=steps, psi0=psi0, return_psi=True, **kw)
    o = orc.solve(p, steps=steps, psi0=psi0)
    return g, o


def _check(p, g, o, steps, field=True, rtol_q=1e-5, atol_scale=None, field_rtol=1e-5):
    oi, oint = _orc_dicts(o)
    ok, rep = compare_qoi(g["qoi"], g["qoi_int"], oi, oint, rtol=rtol_q)
    print(rep)
    assert ok, rep
    if field:
        stages = steps * (2 if p.stepper == I.HEUN else 1)
        okf, repf = compare_field(g["psi"], o["psi"], stages, rtol=field_rtol, atol_scale=atol_scale)
        print("psi:", repf)
        assert okf, repf
        okp, repp = compare_field(g["phi"], o["phi"], stages, rtol=field_rtol,
                                  atol_scale=None if atol_scale is None else atol_scale)
        print("phi:", repp)
        assert okp, repp


BCS = {
    "vacuum": ((I.BC_VACUUM,) * 4, (0.0,) * 4),
    "inflow": ((I.BC_INFLOW, I.BC_INFLOW, I.BC_VACUUM, I.BC_INFLOW), (1.0, 0.5, 0.0, 0.25)),
    "reflect": ((I.BC_REFLECT,) * 4, (0.0,) * 4),
    "mixed": ((I.BC_REFLECT, I.BC_INFLOW, I.BC_INFLOW, I.BC_REFLECT), (0.0, 0.7, 0.3, 0.0)),
}


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("stepper", [I.EULER, I.HEUN])
@pytest.mark.parametrize("bc", list(BCS))
def test_random_state_few_steps(sv, orc, order, stepper, bc):
    """Random materials and a random initial state on a ragged 130 x 37 grid
    (3 x-tiles, partial y-tiles): 2 steps, every field element and QoI."""
    b, g = BCS[bc]
    p = I.random_materials(130, 37, 5, seed=order * 10 + stepper, order=order, stepper=stepper,
                           bc=b, inflow=g, M=32, h=0.05, t_end=1.0)
    psi0 = I.random_state(p, 1234, "smooth")
    g_, o_ = _run_both(sv, orc, p, 2, psi0=psi0)
    _check(p, g_, o_, 2)


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (9, 1), (2, 3), (61, 17), (64, 64), (121, 5), (127, 8),
                                   (128, 9), (129, 7), (257, 16)])
@pytest.mark.parametrize("order", [1, 2])
def test_degenerate_and_tile_edge_shapes(sv, orc, shape, order):
    """Single cells, single rows/columns, and widths and heights at tile
    boundaries (127, 128, 129, 257 columns; 7, 8, 9, 16 rows)."""
    nx, ny = shape
    rects = [(0, 0, nx, ny)]
    if nx >= 3 and ny >= 3:
        rects.append((1, 1, nx - 1, ny - 1))
    p = I.random_materials(nx, ny, 3, seed=nx * 100 + ny, order=order, stepper=I.HEUN,
                           bc=BCS["mixed"][0], inflow=BCS["mixed"][1], M=32, h=0.1, rects=rects)
    psi0 = I.random_state(p, 77, "uniform")
    g_, o_ = _run_both(sv, orc, p, 3, psi0=psi0)
    _check(p, g_, o_, 3)


@pytest.mark.parametrize("rows", [2, 4])
@pytest.mark.parametrize("waves", [4, 8])
@pytest.mark.parametrize("group", [1, 5, 32])
def test_launch_shapes_agree(sv, orc, rows, waves, group):
    """Every compiled launch shape (rows per wave, waves per workgroup) and
    several ordinate-group sizes (ragged last group) give the oracle's answer."""
    p = I.random_materials(73, 70, 4, seed=5, order=2, stepper=I.HEUN, bc=BCS["mixed"][0],
                           inflow=BCS["mixed"][1], M=32, h=0.05)
    psi0 = I.random_state(p, 9, "smooth")
    g_, o_ = _run_both(sv, orc, p, 2, psi0=psi0, group_size=group, rows_per_wave=rows,
                       waves_per_group=waves)
    _check(p, g_, o_, 2)


@pytest.mark.parametrize("rows", [2, 4])
@pytest.mark.parametrize("waves", [4, 8])
@pytest.mark.parametrize("order", [1, 2])
def test_launch_shapes_across_tiles(sv, orc, rows, waves, order):
    """Every launch shape on a grid three tiles wide whose last tile holds
    3 columns, rough initial state: the x-halo cells a tile reads from its
    neighbours' edge records (and from psi's ghost cells on the grid's
    sides) are the oracle's neighbours, for every record height."""
    p = I.random_materials(259, 21, 4, seed=order * 7 + rows + waves, order=order, stepper=I.HEUN,
                           bc=BCS["mixed"][0], inflow=BCS["mixed"][1], M=32, h=0.05,
                           rects=[(0, 0, 259, 21), (120, 3, 131, 18), (250, 1, 258, 20)])
    psi0 = I.random_state(p, 21, "uniform")
    g_, o_ = _run_both(sv, orc, p, 3, psi0=psi0, rows_per_wave=rows, waves_per_group=waves)
    _check(p, g_, o_, 3)


# Rectangles whose boundary faces crowd one tile (the first 128 x 8 tile
# holds about 650 of them: the loader reads that tile's face table from LDS,
# more than four entries per lane), one straddling a tile edge in x and a
# tile row in y, edges on the grid's boundary.
CROWDED_RECTS = [(0, 0, 260, 37), (0, 2, 200, 3), (3, 1, 125, 7), (127, 0, 129, 16)]


@pytest.mark.parametrize("order,stepper", [(1, I.EULER), (2, I.HEUN), (3, I.HEUN)])
def test_crowded_rectangle_faces(sv, orc, order, stepper):
    """Outflow and inflow through many rectangle faces in one tile and across
    tile edges: every QoI and field element against the oracle."""
    p = I.random_materials(260, 37, 4, seed=31 + order, order=order, stepper=stepper, bc=BCS["mixed"][0],
                           inflow=BCS["mixed"][1], M=32, h=0.05, t_end=1.0, rects=CROWDED_RECTS)
    psi0 = I.random_state(p, 55, "smooth")
    g_, o_ = _run_both(sv, orc, p, 2, psi0=psi0)
    _check(p, g_, o_, 2)


def test_no_rectangles(sv, orc):
    p = I.random_materials(40, 30, 3, seed=2, rects=[(0, 0, 40, 30)])
    p = p.replace(rects=np.zeros((0, 4), np.int32), rect_names=[])
    psi0 = I.random_state(p, 4)
    g_, o_ = _run_both(sv, orc, p, 2, psi0=psi0)
    _check(p, g_, o_, 2)


def test_cfg1_lattice_full_run(sv, orc):
    """Lattice 70^2, 32 ordinates, first order, forward Euler, to T = 3.2."""
    p = I.config(1)
    g_, o_ = _run_both(sv, orc, p, None)
    assert g_["nt"] == o_["nt"] == 64 and g_["step"] == 64
    _check(p, g_, o_, 64)


@pytest.mark.parametrize("order", [1, 2])
def test_lattice_heun_full_run(sv, orc, order):
    """Lattice 140^2, 64 ordinates, Heun, to T = 3.2 (128 steps)."""
    p = I.lattice(140, 64, order=order, stepper=I.HEUN)
    g_, o_ = _run_both(sv, orc, p, None)
    _check(p, g_, o_, o_["nt"])


def test_cavity_full_run(sv, orc):
    """Walled cavity 260^2, 64 ordinates, minmod + Heun, to T = 2.6."""
    p = I.cavity(260, 64)
    g_, o_ = _run_both(sv, orc, p, None)
    _check(p, g_, o_, o_["nt"])


def test_homogeneous_closed_form_on_gpu(sv):
    """Reflective box, uniform medium: psi^n from the closed recurrence."""
    Q, sa = 1.3, 0.7
    p = I.homogeneous(nx=70, ny=65, M=32, sigma_a=sa, sigma_s=0.4, q=Q, order=2, stepper=I.HEUN)
    r = sv.solve(p, return_psi=True)
    x = 0.0
    dt = r["dt"]
    for _ in range(r["nt"]):
        x = x * (1 - dt * sa + (dt * sa) ** 2 / 2) + dt * Q * (1 - dt * sa / 2)
    np.testing.assert_allclose(r["psi"], x, rtol=2e-6)
    assert abs(r["balance_residual"]) < 1e-5 * r["qoi_int"]["source"]


def test_balance_residual_small(sv):
    p = I.lattice(70, 32, order=2, stepper=I.HEUN)
    r = sv.solve(p)
    assert abs(r["balance_residual"]) < 1e-5 * r["qoi_int"]["source"], r["balance_residual"]


def test_deterministic(sv):
    p = I.lattice(140, 64, order=2, stepper=I.HEUN)
    a = sv.solve(p, steps=20, return_psi=True)
    b = sv.solve(p, steps=20, return_psi=True)
    assert np.array_equal(a["psi"], b["psi"])
    assert a["qoi_int"] == b["qoi_int"] and a["qoi"] == b["qoi"]


def test_graph_replay_matches_eager(sv):
    p = I.lattice(70, 32, order=1, stepper=I.EULER)
    a = sv.solve(p, return_psi=True)
    b = sv.solve(p, return_psi=True, graph_steps=8)
    assert np.array_equal(a["psi"], b["psi"])
    assert a["qoi_int"] == b["qoi_int"]
    ph = I.lattice(70, 32, order=2, stepper=I.HEUN)
    c = sv.solve(ph, return_psi=True)
    d = sv.solve(ph, return_psi=True, graph_steps=6)
    assert np.array_equal(c["psi"], d["psi"])
    assert c["qoi_int"] == d["qoi_int"]


@pytest.mark.parametrize("order", [1, 2])
def test_bf16_storage_error_bounded(sv, orc, order):
    """BF16 psi storage (stochastic rounding on store, FP32 math): each stored
    value carries a relative rounding error below one bfloat16 ulp, 2^-8 (half
    that for round-to-nearest, which is biased), so after four stages the
    field error stays within a few 2^-8 of the local magnitude."""
    p = I.random_materials(130, 37, 5, seed=3, order=order, stepper=I.HEUN, bc=BCS["mixed"][0],
                           inflow=BCS["mixed"][1], M=32, psi_dtype="bf16")
    psi0 = I.random_state(p, 5, "smooth")  # exact in bf16
    g_, o_ = _run_both(sv, orc, p, 2, psi0=psi0)
    okf, rep = compare_field(g_["psi"], o_["psi"], 4, rtol=4 * 2.0 ** -8, atol_scale=2.0 ** -8)
    print("bf16 psi:", rep)
    assert okf, rep


def test_full_size_lattice700_random_state(sv, orc):
    """The benchmark workload (700^2 lattice, 256 ordinates, minmod, Heun) in
    its default launch shape: one step from a random state, sampled field
    values and every QoI against the oracle."""
    p = I.config(2)
    psi0 = I.random_state(p, 2024, "smooth")
    g_, o_ = _run_both(sv, orc, p, 1, psi0=psi0)
    oi, oint = _orc_dicts(o_)
    ok, rep = compare_qoi(g_["qoi"], g_["qoi_int"], oi, oint)
    print(rep)
    assert ok, rep
    rng = np.random.Generator(np.random.PCG64(0))
    idx = tuple(rng.integers(0, s, 20000) for s in o_["psi"].shape)
    okf, repf = compare_field(g_["psi"][idx], o_["psi"][idx], 2)
    print("sampled psi:", repf)
    assert okf, repf
    okp, repp = compare_field(g_["phi"], o_["phi"], 2)
    print("phi:", repp)
    assert okp, repp


def test_full_size_cavity1300_random_state(sv, orc):
    """The walled-cavity configuration at full size (1300^2 cells, 512
    ordinates, minmod, Heun, inflow through the west side; 3.5 GB per psi
    buffer, far above the 256 MB Infinity Cache) in its default launch shape:
    one step from a random state, sampled field values, phi and every QoI
    against the oracle."""
    p = I.config(3)
    psi0 = I.random_state(p, 1300, "smooth")
    g_, o_ = _run_both(sv, orc, p, 1, psi0=psi0)
    del psi0
    oi, oint = _orc_dicts(o_)
    ok, rep = compare_qoi(g_["qoi"], g_["qoi_int"], oi, oint)
    print(rep)
    assert ok, rep
    rng = np.random.Generator(np.random.PCG64(1))
    idx = tuple(rng.integers(0, s, 50000) for s in o_["psi"].shape)
    okf, repf = compare_field(g_["psi"][idx], o_["psi"][idx], 2)
    print("sampled psi:", repf)
    assert okf, repf
    okp, repp = compare_field(g_["phi"], o_["phi"], 2)
    print("phi:", repp)
    assert okp, repp


@pytest.mark.parametrize("order", [1, 2])
def test_hohlraum_random_state_few_steps(sv, orc, order):
    """The Hohlraum layout (five materials, sigma_t up to 100, inflow through
    both x sides): every element of psi and phi and every QoI after two Heun
    steps from a random state."""
    p = I.hohlraum(130, 32, order=order)
    psi0 = I.random_state(p, 77, "smooth")
    g, o = _run_both(sv, orc, p, 2, psi0=psi0)
    _check(p, g, o, 2)


def test_hohlraum260_full_run_matches_golden(sv):
    """Full Hohlraum solve (260^2 cells, 256 ordinates, minmod, Heun, 1040
    steps to T = 2.6) against the oracle's QoIs stored by
    tests/golden/make_oracle_goldens.py."""
    path = os.path.join(GOLDEN, "oracle_hohlraum260_M256_heun2.json")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    with open(path) as f:
        gold = json.load(f)
    p = I.hohlraum(260, 256)
    r = sv.solve(p)
    ok, rep = compare_qoi(r["qoi"], r["qoi_int"], gold["qoi"], gold["qoi_int"], per_qoi=True)
    print(rep)
    assert ok, rep


def test_lattice700_full_run_matches_golden(sv):
    """Full 640-step solve of the benchmark workload against the oracle's QoIs
    stored by tests/golden/make_oracle_goldens.py."""
    path = os.path.join(GOLDEN, "oracle_lattice700_M256_heun2.json")
    if not os.path.exists(path):
        pytest.skip("golden not generated")
    with open(path) as f:
        gold = json.load(f)
    p = I.config(2)
    r = sv.solve(p)
    ok, rep = compare_qoi(r["qoi"], r["qoi_int"], gold["qoi"], gold["qoi_int"], per_qoi=True)
    print(rep)
    assert ok, rep


@pytest.mark.parametrize("N,order", [(5, 2), (22, 2), (22, 1), (5, 3), (22, 3)])
def test_tessellation_quadrature_random_state(sv, orc, N, order):
    """The paper's tessellation quadrature (M = 4 N^2: 100, and 1936 at the
    finest N = 22, where ordinate groups run to ~242 ordinates): every element
    of psi and phi and every QoI after two Heun steps from a random state on a
    ragged lattice grid with reflective and inflow sides, for every order
    (at order 3 the reflective ghosts of every ordinate come from its
    mirror in this quadrature)."""
    p = I.lattice(71, order=order, stepper=I.HEUN, quad=I.tessellation_quadrature(N),
                  bc=(I.BC_REFLECT, I.BC_INFLOW, I.BC_REFLECT, I.BC_VACUUM))
    p = p.replace(inflow=(0.0, 0.6, 0.0, 0.0))
    psi0 = I.random_state(p, 31 + N)
    g, o = _run_both(sv, orc, p, 2, psi0=psi0)
    _check(p, g, o, 2)


def test_full_size_tessellation22_random_state(sv, orc):
    """The 700^2 lattice with the tessellation quadrature at N = 22 (1936
    ordinates, 3.8 GB per psi buffer) in the launch shape the bench times:
    one Heun step from a random state, sampled psi, all of phi and every QoI
    against the oracle."""
    p = I.lattice(700, order=2, stepper=I.HEUN, quad=I.tessellation_quadrature(22))
    psi0 = I.random_state(p, 2222, "smooth")
    g_, o_ = _run_both(sv, orc, p, 1, psi0=psi0)
    del psi0
    oi, oint = _orc_dicts(o_)
    ok, rep = compare_qoi(g_["qoi"], g_["qoi_int"], oi, oint)
    print(rep)
    assert ok, rep
    rng = np.random.Generator(np.random.PCG64(4))
    idx = tuple(rng.integers(0, s, 50000) for s in o_["psi"].shape)
    okf, repf = compare_field(g_["psi"][idx], o_["psi"][idx], 2)
    print("sampled psi:", repf)
    assert okf, repf
    okp, repp = compare_field(g_["phi"], o_["phi"], 2)
    print("phi:", repp)
    assert okp, repp


def test_full_size_cavity_share_of_eight(sv, orc):
    """One GPU's share of an 8-way ordinate split of the full-size cavity:
    1300^2 cells with 64 ordinates, in its default launch shape (2 groups of
    32 ordinates). One Heun step from a smooth random state: every QoI,
    sampled psi and all of phi against the oracle."""
    p = I.cavity(1300, 64)
    info = sv.plan_info(p)
    assert (info["group_size"], info["group_size_average"]) == (32, 32)
    psi0 = I.random_state(p, 77, "smooth")
    g_, o_ = _run_both(sv, orc, p, 1, psi0=psi0)
    oi, oint = _orc_dicts(o_)
    ok, rep = compare_qoi(g_["qoi"], g_["qoi_int"], oi, oint)
    print(rep)
    assert ok, rep
    rng = np.random.Generator(np.random.PCG64(8))
    idx = tuple(rng.integers(0, s, 20000) for s in o_["psi"].shape)
    okf, repf = compare_field(g_["psi"][idx], o_["psi"][idx], 2)
    print("sampled psi:", repf)
    assert okf, repf
    okp, repp = compare_field(g_["phi"], o_["phi"], 2)
    print("phi:", repp)
    assert okp, repp
