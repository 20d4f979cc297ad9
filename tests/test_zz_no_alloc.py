"""sn_plan_bind_static: a plan whose scratch is the library's own device area
(for callers that cannot allocate device memory) gives the same results as the
same plan bound to caller scratch, call after call, the second call with a
smaller input than the first (the area keeps what the last plan left in it).
Through the C ABI (ctypes), on the GPU."""

import numpy as np
import pytest

from paper_2505_17284_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17284_amd import solver

    return solver


def _run(solver, p, static, steps=None):
    plan = solver.Plan(p, static_scratch=static)
    try:
        plan.run(steps)
        mid = plan.qoi()
        plan.run()
        return dict(mid=mid, end=plan.qoi(), psi=plan.psi(), phi=plan.phi())
    finally:
        plan.close()


def _same(a, b, what):
    assert np.array_equal(a["psi"], b["psi"]), f"{what}: psi differs"
    assert np.array_equal(a["phi"], b["phi"]), f"{what}: phi differs"
    for k in ("mid", "end"):
        assert a[k]["qoi"] == b[k]["qoi"], f"{what}: {k} QoIs differ"
        assert a[k]["qoi_int"] == b[k]["qoi_int"], f"{what}: {k} integrated QoIs differ"
        assert a[k]["step"] == b[k]["step"]


def test_static_scratch_matches_caller_scratch_twice(solver):
    mixed = (I.BC_REFLECT, I.BC_INFLOW, I.BC_INFLOW, I.BC_REFLECT)
    big = I.lattice(140, 64, order=2, stepper=I.HEUN, t_end=0.8, name="lattice140_M64_short")
    small = I.random_materials(61, 17, 4, seed=1, M=32, bc=mixed, inflow=(0.0, 0.7, 0.3, 0.0), t_end=0.3)
    for p in (big, small):  # the second call's input is smaller
        print(f"[case] {p.name}: static vs caller scratch", flush=True)
        ref = _run(solver, p, static=False, steps=5)
        got = _run(solver, p, static=True, steps=5)
        _same(got, ref, p.name)
        assert got["end"]["step"] == solver.plan_info(p)["n_steps"]


def test_static_scratch_bf16_and_euler(solver):
    for p in (I.lattice(70, 32, order=1, stepper=I.EULER, name="lattice70_euler"),
              I.lattice(70, 32, order=2, stepper=I.HEUN, psi_dtype="bf16", name="lattice70_bf16")):
        print(f"[case] {p.name}: static vs caller scratch", flush=True)
        _same(_run(solver, p, static=True, steps=3), _run(solver, p, static=False, steps=3), p.name)


def test_one_plan_at_a_time(solver):
    from paper_2505_17284_amd._lib import SN_ERR_BUSY, SnError

    p = I.lattice(70, 32, order=2, stepper=I.HEUN)
    a = solver.Plan(p, static_scratch=True)
    try:
        with pytest.raises(SnError) as ei:
            solver.Plan(p, static_scratch=True)
        assert ei.value.status == SN_ERR_BUSY
    finally:
        a.close()
    # destroying the holder frees the area
    b = solver.Plan(p, static_scratch=True)
    b.close()
