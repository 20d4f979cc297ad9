"""Per-QoI error of the stored-psi precisions against the FP64 oracle.

The full lattice benchmark (700^2 cells, 256 ordinates, minmod, Heun, 640
steps to T = 3.2) is solved with FP32 and with BF16 psi storage (FP32
arithmetic in both), and the full walled cavity (1300^2 cells, 64
ordinates, 5200 steps) with BF16 storage; every instantaneous and
time-integrated QoI is compared with the oracle's values stored by
tests/golden/make_oracle_goldens.py.
FP32 is held to the 1e-5 relative target. BF16 keeps 8 significant bits per
stored value (stochastic rounding, so without bias); it is held to 1e-2
relative or 1e-5 of the problem's scale (the largest QoI of the same kind),
whichever is larger: the outflow through the outer boundary is four orders
below the mass and carries the storage noise of the nearly empty edge cells.
Run with -s to see the table.
"""

import json
import os

import pytest

from paper_2505_17284_amd import inputs as I
from tests.parity import compare_qoi

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_lattice700_M256_heun2.json")
BOUND = {"f32": 1e-5, "bf16": 1e-2}


@pytest.fixture(scope="module")
def sv():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17284_amd import solver

    return solver


CAVITY_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_cavity1300_M64_heun2.json")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_lattice700_full_run_error_per_qoi(sv, dtype):
    _full_run_error_per_qoi(sv, GOLDEN, I.config(2), dtype)


def test_cavity1300_M64_bf16_full_run_error_per_qoi(sv):
    """The walled cavity at full grid and length (1300^2, 5200 Heun steps),
    one GPU's 64-ordinate share, BF16 storage, against the stored oracle run
    (FP32 storage of the same run: tests/test_gpu_fullrun.py)."""
    _full_run_error_per_qoi(sv, CAVITY_GOLDEN, I.cavity(1300, 64, name="cavity1300_M64_heun2"), "bf16")


def _full_run_error_per_qoi(sv, golden, problem, dtype):
    if not os.path.exists(golden):
        pytest.skip("golden not generated")
    with open(golden) as f:
        gold = json.load(f)
    p = problem.replace(psi_dtype=dtype)
    print(f"[case] {p.name} psi {dtype}", flush=True)
    r = sv.solve(p)
    assert r["nt"] == gold["nt"]
    print(f"| storage | QoI | oracle (FP64) | GPU | relative error |")
    for kind, g, o in (("at T", r["qoi"], gold["qoi"]), ("integrated", r["qoi_int"], gold["qoi_int"])):
        for name, ov in o.items():
            gv = g[name]
            rel = abs(gv - ov) / abs(ov) if ov else abs(gv - ov)
            print(f"| {dtype} | {name} {kind} | {ov:.10g} | {gv:.10g} | {rel:.2e}{'' if ov else ' (abs)'} |")
    if dtype == "f32":
        ok, rep = compare_qoi(r["qoi"], r["qoi_int"], gold["qoi"], gold["qoi_int"], rtol=BOUND[dtype],
                              per_qoi=True)
        assert ok, rep
        return
    for g, o in ((r["qoi"], gold["qoi"]), (r["qoi_int"], gold["qoi_int"])):
        scale = max(abs(v) for v in o.values())
        for name, ov in o.items():
            err = abs(g[name] - ov)
            assert err <= max(BOUND[dtype] * abs(ov), 1e-5 * scale), (name, g[name], ov)
