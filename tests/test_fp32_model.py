"""What FP32 arithmetic alone does to the scheme (sets long-run field tolerances).

The lattice at 140^2 with 64 ordinates, minmod and Heun has one spot (the
corner of the source block, one mirror pair of ordinates) where the FP32 state
drifts from the FP64 result by ~1e-4 of the peak within 128 steps while the
field as a whole stays within ~2e-7 in relative L1. A float64 run of the same
NumPy model reproduces the oracle, so the drift is arithmetic, not a model
difference. The GPU parity tests for long runs use the bounds checked here.
"""

import numpy as np
import pytest

from paper_2505_17284_amd import inputs as I
from tests import fp32_model as FM
from tests.parity import LONG_L1, LONG_FRAC, LONG_CAP


@pytest.fixture(scope="module")
def case(orc):
    p = I.lattice(140, 64, order=2, stepper=I.HEUN)
    nt, dt = orc.num_steps(p)
    ref = orc.solve(p, steps=128)["psi"]
    return p, dt, ref


def test_float64_model_reproduces_oracle(orc):
    p = I.lattice(70, 32, order=2, stepper=I.HEUN)
    nt, dt = orc.num_steps(p)
    ref = orc.solve(p, steps=20)["psi"]
    got = FM.run(p, 20, dt, np.float64)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_float32_drift_within_long_run_bounds(case):
    p, dt, ref = case
    got = FM.run(p, 128, dt, np.float32)
    err = np.abs(got - ref)
    peak = np.abs(ref).max()
    l1 = err.sum() / np.abs(ref).sum()
    tight = 1e-5 * np.abs(ref) + 2e-7 * (2 * 128 + 2) * peak
    frac = np.mean(err > tight)
    print(f"fp32 model after 128 steps: max {err.max() / peak:.2e} of peak, L1 {l1:.2e}, frac {frac:.2e}")
    assert err.max() > 1e-5 * peak  # the drift is real: per-element 1e-5 is out of reach
    assert l1 <= LONG_L1 / 4 and frac <= LONG_FRAC / 4 and err.max() <= LONG_CAP * peak / 4
