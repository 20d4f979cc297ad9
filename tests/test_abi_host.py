"""The C ABI without a GPU: the library loads, exports every declared entry
point, and validates problem statements on the host."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2505_17284_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2505_17284_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2505_17284_amd import build

        build.build()
    return _lib


def _declared():
    with open(os.path.join(ROOT, "include", "snrt.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sn_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 15
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), f"{n} declared in snrt.h but not exported"
    assert sorted(L.EXPORTED) == names


def test_status_strings(L):
    lib = L.lib()
    for s in range(8):
        assert lib.sn_status_str(s)


def _create(L, p, **kw):
    m = L.MarshalledProblem(p)
    for k, v in kw.items():
        setattr(m.struct, k, v)
    h = ctypes.c_void_p()
    st = L.lib().sn_plan_create(ctypes.byref(m.struct), ctypes.byref(h))
    if st == 0:
        L.lib().sn_plan_destroy(h)
    return st, L.lib().sn_last_error().decode()


def test_valid_problems_accepted(L):
    for p in (I.config(1), I.config(2), I.config(3), I.uq_instance(0), I.beam(), I.homogeneous()):
        st, msg = _create(L, p)
        assert st == 0, msg


@pytest.mark.parametrize("field,value,needle", [
    ("cfl", 0.0, "cfl"), ("cfl", float("nan"), "cfl"), ("t_end", -1.0, "t_end"),
    ("h", 0.0, "cell size"), ("nx", 0, "grid"), ("order", 4, "order"), ("stepper", 2, "stepper"),
    ("n_tallies", 9, "n_tallies"), ("n_rects", 5, "n_rects"), ("psi_dtype", 7, "psi_dtype"),
    ("M", 0, "M ="), ("n_regions", 0, "n_regions"),
])
def test_invalid_statements_rejected(L, field, value, needle):
    st, msg = _create(L, I.config(1), **{field: value})
    assert st == L.SN_ERR_INVALID and needle in msg, msg


def test_semantic_rejections(L):
    p = I.config(1)
    bad_w = p.quad.w.copy() * 1.001
    q = I.Quadrature(p.quad.mu, p.quad.xi, p.quad.eta, bad_w, p.quad.mirror_x, p.quad.mirror_y, 4, 8)
    st, msg = _create(L, p.replace(quad=q))
    assert st == L.SN_ERR_INVALID and "2 pi" in msg
    # reflective walls need exact mirror partners
    mx = p.quad.mirror_x.copy()
    mx[0], mx[1] = mx[1], mx[0]
    q2 = I.Quadrature(p.quad.mu, p.quad.xi, p.quad.eta, p.quad.w, mx, p.quad.mirror_y, 4, 8)
    st, msg = _create(L, p.replace(quad=q2, bc=(I.BC_REFLECT,) * 4))
    assert st == L.SN_ERR_INVALID and "mirror" in msg
    st, _ = _create(L, p.replace(quad=q2))  # not needed without reflective sides
    assert st == 0
    reg = p.region.copy()
    reg[3, 4] = 7
    st, msg = _create(L, p.replace(region=reg))
    assert st == L.SN_ERR_INVALID and "region id" in msg
    st, msg = _create(L, p.replace(rects=np.array([(0, 0, 71, 70)], np.int32)))
    assert st == L.SN_ERR_INVALID and "rect" in msg
    st, msg = _create(L, p.replace(sigma_a=np.array([0.0, -1.0, 0.0])))
    assert st == L.SN_ERR_INVALID and "cross-sections" in msg
    tal = np.array([0, 1, 5], np.uint8)
    st, msg = _create(L, p.replace(tally=tal))
    assert st == L.SN_ERR_INVALID and "tally" in msg


def test_time_steps_agree_with_oracle(L, orc):
    """Library and oracle derive N_t and dt independently from (T, CFL, h)."""
    from paper_2505_17284_amd import solver

    for p in (I.config(1), I.config(2), I.config(3), I.lattice(100, 32), I.uq_instance(3),
              I.cavity(333, 32)):
        info = solver.plan_info(p)
        nt, dt = orc.num_steps(p)
        assert info["n_steps"] == nt and info["dt"] == dt, (p.name, info["n_steps"], nt)


def test_buffer_sizes(L):
    from paper_2505_17284_amd import solver

    info = solver.plan_info(I.config(2))
    assert info["pitch"] >= 700 and info["pitch"] % 16 == 0
    assert info["psi_bytes"] >= 256 * 700 * info["pitch"] * 4
    assert info["psi_bytes"] % 256 == 0 and info["scratch_bytes"] % 256 == 0
    bf = solver.plan_info(I.config(2).replace(psi_dtype="bf16"))
    assert bf["psi_bytes"] < info["psi_bytes"] * 0.55  # BF16 rows start one 128-byte line in too


def test_calls_in_wrong_order_fail_cleanly(L):
    p = I.config(1)
    m = L.MarshalledProblem(p)
    h = ctypes.c_void_p()
    lib = L.lib()
    assert lib.sn_plan_create(ctypes.byref(m.struct), ctypes.byref(h)) == 0
    try:
        assert lib.sn_plan_run(h, 1, None) == L.SN_ERR_STATE
        q = L.SnQoi()
        assert lib.sn_plan_qoi(h, ctypes.byref(q), None) == L.SN_ERR_STATE
        assert lib.sn_plan_bind(h, None, None, None) == L.SN_ERR_INVALID
        assert lib.sn_plan_bind(h, ctypes.c_void_p(256), ctypes.c_void_p(512), ctypes.c_void_p(1024)) \
            == L.SN_ERR_INVALID  # overlapping
        assert lib.sn_plan_use_graph(h, 3) == L.SN_ERR_INVALID
    finally:
        lib.sn_plan_destroy(h)


def _create_probes(L, p, probes):
    m = L.MarshalledProblem(p, probes=probes)
    h = ctypes.c_void_p()
    st = L.lib().sn_plan_create(ctypes.byref(m.struct), ctypes.byref(h))
    if st == 0:
        L.lib().sn_plan_destroy(h)
    return st, L.lib().sn_last_error().decode()


def test_probe_statements(L):
    """Probe lists are validated on the host; a tile of 128 x 8 cells (the
    default launch shape) takes at most 64 loader lanes of 8 cells, a lane's
    cells all of one probe."""
    from paper_2505_17284_amd import hohlraum

    p = I.hohlraum(260, 32)
    pr = hohlraum.probe_cells(p)
    assert _create_probes(L, p, pr)[0] == 0
    bad = dict(pr, n_probes=L.MAX_PROBES + 1)
    st, msg = _create_probes(L, p, bad)
    assert st == L.SN_ERR_INVALID and "n_probes" in msg, msg
    cells = pr["cells"].copy()
    cells["probe"][0] = 4
    st, msg = _create_probes(L, p, dict(pr, cells=cells))
    assert st == L.SN_ERR_INVALID and "probe 4" in msg, msg
    cells = pr["cells"].copy()
    cells["cell"][0] = 260 * 260
    st, msg = _create_probes(L, p, dict(pr, cells=cells))
    assert st == L.SN_ERR_INVALID and "cell index" in msg, msg

    # capacity of one tile: columns 0..127, rows 0..7
    def tile_cells(counts):
        recs, c = [], 0
        for q, n in enumerate(counts):
            for _ in range(n):
                recs.append(((c // 128) * 260 + c % 128, q, 1.0 / n))
                c += 1
        return dict(n_probes=len(counts), n_windows=3, cells=np.array(recs, dtype=L.PROBE_CELL))

    assert _create_probes(L, p, tile_cells([512]))[0] == 0          # 64 lanes of 8
    # 505 cells need 64 lanes of 8 (one slot free); the other probe needs a lane of its own
    st, msg = _create_probes(L, p, tile_cells([505, 7]))
    assert st == L.SN_ERR_UNSUPPORTED and "probe cells in the tile" in msg, msg
    st, msg = _create_probes(L, p, tile_cells([513]))
    assert st == L.SN_ERR_UNSUPPORTED, msg
    assert _create_probes(L, p, tile_cells([448] + [8] * 7))[0] == 0  # 56 + 7 lanes
    # a ball of radius 30 h fits wherever it sits
    q = I.hohlraum(1300, 32)
    big = hohlraum.probe_cells(q, centres=((0.0, 0.0), (0.3, -0.2)), r=30 * q.h)
    assert _create_probes(L, q, big)[0] == 0


def test_default_launch_shapes(L):
    """The default launch shapes of the measured workloads (host only): with
    FP32 storage eight waves per workgroup and 32 ordinates per group on grids
    of 10^6 cells or more (the cavity and one GPU's 64-ordinate share of it)
    and on 4 10^5 or more with 512 ordinates; otherwise four waves, 16
    ordinates per group where 32 would give 1,000 to 5,000 workgroups (the
    benchmark lattice, 560^2 at 128 and 256 ordinates), 32 with the averaging
    stage halved above that at 256 ordinates or more (560^2 x 512), fewer on
    grids too small to fill the GPU otherwise; no such change with the
    Venkatakrishnan limiter; BF16 storage keeps four waves and groups of 64."""
    from paper_2505_17284_amd import solver

    def g(p):
        i = solver.plan_info(p)
        return i["group_size"], i["group_size_average"], i["rows_per_wave"], i["waves_per_group"]

    assert g(I.config(2)) == (16, 16, 2, 4)
    assert g(I.config(2).replace(psi_dtype="bf16")) == (64, 64, 2, 4)
    assert g(I.config(2).replace(order=3)) == (32, 32, 2, 4)
    assert g(I.config(3)) == (32, 32, 2, 8)
    assert g(I.config(3).replace(psi_dtype="bf16")) == (64, 64, 2, 4)
    assert g(I.cavity(1300, 64)) == (32, 32, 2, 8)
    assert g(I.lattice(140, 64, order=2, stepper=I.HEUN)) == (8, 8, 2, 4)
    assert g(I.lattice(140, 256, order=2, stepper=I.HEUN)) == (16, 16, 2, 4)
    assert g(I.lattice(560, 128, order=2, stepper=I.HEUN)) == (16, 16, 2, 4)
    assert g(I.lattice(560, 256, order=2, stepper=I.HEUN)) == (16, 16, 2, 4)
    assert g(I.lattice(560, 512, order=2, stepper=I.HEUN)) == (32, 16, 2, 4)
    assert g(I.lattice(700, 512, order=2, stepper=I.HEUN)) == (32, 32, 2, 8)


def test_static_scratch_rejects_what_it_cannot_hold(L):
    """sn_plan_bind_static refuses NULL buffers and plans whose scratch exceeds
    SN_STATIC_SCRATCH_BYTES before touching the device."""
    lib = L.lib()
    big = I.config(3)  # 1300^2 x 512: more scratch than the static area holds
    m = L.MarshalledProblem(big)
    h = ctypes.c_void_p()
    assert lib.sn_plan_create(ctypes.byref(m.struct), ctypes.byref(h)) == 0
    try:
        info = L.SnPlanInfo()
        assert lib.sn_plan_get_info(h, ctypes.byref(info)) == 0
        assert info.scratch_bytes > L.STATIC_SCRATCH_BYTES
        assert lib.sn_plan_bind_static(h, None, None) == L.SN_ERR_INVALID
        assert lib.sn_plan_bind_static(h, ctypes.c_void_p(256), ctypes.c_void_p(1 << 40)) == L.SN_ERR_UNSUPPORTED
        assert "SN_STATIC_SCRATCH_BYTES" in lib.sn_last_error().decode()
    finally:
        lib.sn_plan_destroy(h)


def test_crowded_rectangle_faces_accepted(L):
    """Plan creation lists every rectangle-boundary face per tile with the
    ring-slot offsets of the cells its trace needs, and rejects the plan if
    one of those cells is not staged with the tile: rectangles crowding one
    tile, straddling tile edges and lying on the grid's boundary, at every
    order, storage type and launch shape."""
    from paper_2505_17284_amd import solver

    rects = [(0, 0, 260, 37), (0, 2, 200, 3), (3, 1, 125, 7), (127, 0, 129, 16)]
    edge = [(259, 0, 260, 37), (0, 36, 260, 37), (128, 8, 129, 9), (0, 0, 1, 1)]
    for rs in (rects, edge):
        for order in (1, 2, 3):
            for dtype in ("f32", "bf16"):
                p = I.random_materials(260, 37, 4, seed=3, order=order, M=32, rects=rs, psi_dtype=dtype)
                for rows, waves in ((2, 4), (4, 4), (2, 8), (4, 8)):
                    info = solver.plan_info(p, rows_per_wave=rows, waves_per_group=waves)
                    assert info["scratch_bytes"] > 0
