"""Error and reproducibility conventions of the C ABI on the GPU.

* A QoI that becomes NaN or infinite makes sn_plan_qoi return
  SN_ERR_NONFINITE (with the QoIs filled in and nonfinite = 1).
* One failing request does not disturb the others: in a batch and in the
  serving loop the other members finish bit-identical to their solves alone,
  and only the failing one carries nonfinite = 1.
* Reading QoIs mid-run is not a stage: a BF16 plan whose QoIs are read
  between runs ends bit-identical to one left alone (the stochastic-rounding
  bits follow the stage count).

The non-finite values are plain floating-point overflow of a numerically
unstable but valid problem statement (or an infinite initial value), not a
device fault: every kernel runs to its normal end.
"""

import numpy as np
import pytest

from paper_2505_17284_amd import inputs as I

pytestmark = pytest.mark.gpu

SN_ERR_NONFINITE = 5


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17284_amd import batch, serve, solver

    return batch, serve, solver


def diverging(seed=5, nx=40, ny=30):
    """Valid inputs whose explicit Heun step is unstable: dt sigma_t = 10 (h = 0.05,
    CFL 0.5) multiplies the state by about 41 per step, so FP32 overflows within
    about 25 of its 80 steps and the QoIs turn infinite, then NaN."""
    p = I.random_materials(nx, ny, 3, seed=seed, M=32, t_end=2.0)
    return p.replace(sigma_a=np.full(3, 400.0), name=f"diverging_{nx}x{ny}_s{seed}")


def good_mix():
    refl = (I.BC_REFLECT,) * 4
    return [
        I.lattice(70, 32, order=2, stepper=I.HEUN),
        I.random_materials(61, 17, 4, seed=1, M=64, t_end=0.3, bc=(I.BC_REFLECT, I.BC_INFLOW, I.BC_INFLOW,
                                                                     I.BC_REFLECT), inflow=(0.0, 0.7, 0.3, 0.0)),
        I.random_materials(130, 37, 5, seed=2, M=32, bc=refl, t_end=0.45, rects=[(0, 0, 130, 37)]),
    ]


def test_infinite_initial_value_reports_nonfinite(gpu):
    _, _, solver = gpu
    from paper_2505_17284_amd._lib import SnError

    p = I.lattice(70, 32, order=2, stepper=I.HEUN, name="lattice70_inf_psi0")
    psi0 = np.zeros((p.M, p.ny, p.nx), dtype=np.float32)
    psi0[3, 20, 30] = np.inf
    print(f"[case] {p.name}: psi0 holds one +inf, 2 steps", flush=True)
    plan = solver.Plan(p, psi0=psi0)
    try:
        plan.run(2)
        with pytest.raises(SnError) as ei:
            plan.qoi()
        assert ei.value.status == SN_ERR_NONFINITE
        r = plan.qoi(allow_nonfinite=True)
        assert r["nonfinite"]
        assert not np.isfinite(r["qoi"]["mass"])
    finally:
        plan.close()


def test_finite_run_reports_ok(gpu):
    _, _, solver = gpu
    p = I.lattice(70, 32, order=2, stepper=I.HEUN)
    r = solver.solve(p, steps=4)
    assert not r["nonfinite"]


def test_diverging_solve_reports_nonfinite(gpu):
    _, _, solver = gpu
    from paper_2505_17284_amd._lib import SnError

    p = diverging()
    print(f"[case] {p.name} to T", flush=True)
    plan = solver.Plan(p)
    try:
        plan.run()
        with pytest.raises(SnError) as ei:
            plan.qoi()
        assert ei.value.status == SN_ERR_NONFINITE
        assert plan.qoi(allow_nonfinite=True)["step"] == plan.n_steps
    finally:
        plan.close()


def _same(a, b, what):
    assert np.array_equal(a["psi"], b["psi"]), f"{what}: psi differs"
    assert a["qoi"] == b["qoi"], f"{what}: QoIs differ"
    assert a["qoi_int"] == b["qoi_int"], f"{what}: integrated QoIs differ"


@pytest.mark.parametrize("use_graph", [False, True])
def test_nonfinite_member_is_isolated_in_a_batch(gpu, use_graph):
    batch, _, solver = gpu
    good = good_mix()
    alone = []
    for p in good:
        print(f"[case] alone {p.name}", flush=True)
        alone.append(solver.solve(p, return_psi=True, rows_per_wave=2, waves_per_group=4))
    bad = diverging()
    print(f"[case] batch with {bad.name}, graph={use_graph}", flush=True)
    b = batch.Batch(max_instances=8, steps_per_run=5, use_graph=use_graph)
    try:
        probs = good[:2] + [bad] + good[2:]
        slots = [b.admit(p) for p in probs]
        while b.unfinished():
            b.run()
        res = [b.result(s, psi=True, allow_nonfinite=True) for s in slots]
        for p, r in zip(probs, res):
            assert r["nonfinite"] == (p is bad), p.name
        for p, r, a in zip(good, res[:2] + res[3:], alone):
            _same(r, a, p.name)
    finally:
        b.close()


def test_nonfinite_request_is_isolated_in_serving(gpu):
    _, serve, solver = gpu
    good = good_mix()
    bad = diverging()
    reqs = [(0.0, good[0]), (0.0, bad), (0.01, good[1]), (0.02, good[2])]
    print("[case] serving mix with one diverging request", flush=True)
    rec, tot = serve.serve(reqs, int(8e9), max_instances=8, steps_per_run=8, policy="srpt")
    by_name = {r["name"]: r for r in rec}
    assert by_name[bad.name]["nonfinite"]
    for p in good:
        r = by_name[p.name]
        assert not r["nonfinite"], p.name
        a = solver.solve(p, rows_per_wave=2, waves_per_group=4)
        assert r["qoi_int"] == a["qoi_int"], p.name


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_midrun_qoi_reads_do_not_change_the_result(gpu, dtype):
    _, _, solver = gpu
    p = I.lattice(70, 32, order=2, stepper=I.HEUN, psi_dtype=dtype, name=f"lattice70_{dtype}_polled")
    print(f"[case] {p.name}: 12 steps with and without QoI reads every 3", flush=True)
    plain = solver.Plan(p)
    polled = solver.Plan(p)
    try:
        plain.run(12)
        for _ in range(4):
            polled.run(3)
            polled.qoi()
        a, b = plain.psi(), polled.psi()
        assert np.array_equal(a, b), f"psi differs after mid-run QoI reads (max {np.abs(a - b).max()})"
        qa, qb = plain.qoi(), polled.qoi()
        assert qa["qoi_int"] == qb["qoi_int"]
    finally:
        plain.close()
        polled.close()
