"""The oracle's lattice QoIs against the paper's own table (Sec. 6.1, lattice
reference table), as a loose plausibility check, not parity: the paper solves
on unstructured triangles with the tessellation quadrature, the
Venkatakrishnan limiter and CFL 0.7; the oracle on square cells with a
product quadrature, minmod and CFL 0.5.

The series is the benchmark scheme (minmod, Heun) at 70^2 x 32, 140^2 x 64
and the stored 700^2 x 256 oracle solve (tests/golden).

* QoI-3, QoI-4, QoI-5 (absorption in B at T and over [0, T], mass at T,
  Sec. 3.1.2) converge onto the table: within 1% from 140^2 on.
* QoI-1 and QoI-2 at l = 1.5 (outflow through the boundary of S_l at T and
  over [0, T]), evaluated as printed in Sec. 3.1.2 (the gross outflow
  over gamma_l^+ with the measure d mu d phi of P), come out twice the
  table: the ratio rises under refinement towards 2 (1.93, 1.97, 1.98 at T)
  and is the same at T and over [0, T], so the table holds half of the
  printed functional. No passage of the paper halves it; the library and the
  oracle keep the functional as printed, and this test records the factor.
  The other readings tried (the net outflow, S_l of half-width l / 2, the
  corner [0, l]^2 of the shifted domain) are far off.
* At l = 2.5 the table's values are about 10^-4 of those at l = 1.5, with
  QoI-1 > QoI-2; the printed functional on the oracle's solution is several
  hundred times larger. The test records that gap; no reading of S_l
  reproduces the table there.
"""

import json
import os

import pytest

from paper_2505_17284_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def _table():
    with open(os.path.join(HERE, "golden", "paper_lattice_table.json")) as f:
        t = json.load(f)
    return {k: v["mean"] for k, v in t.items() if not k.startswith("_")}


@pytest.fixture(scope="module")
def series(orc):
    out = []
    for n, M in ((70, 32), (140, 64)):
        r = orc.solve(I.lattice(n, M, order=2, stepper=I.HEUN))
        out.append((n, dict(zip(r["names"], map(float, r["qoi"]))), dict(zip(r["names"], map(float, r["qoi_int"])))))
    with open(os.path.join(HERE, "golden", "oracle_lattice700_M256_heun2.json")) as f:
        g = json.load(f)
    out.append((700, g["qoi"], g["qoi_int"]))
    return out


def test_absorption_and_mass_converge_onto_the_table(series):
    tab = _table()
    for n, q, qi in series:
        rel = {"QoI-3": q["abs:B"] / tab["QoI-3"] - 1, "QoI-4": qi["abs:B"] / tab["QoI-4"] - 1,
               "QoI-5": q["mass"] / tab["QoI-5"] - 1}
        print(n, {k: f"{v:+.2e}" for k, v in rel.items()})
        if n >= 140:
            assert all(abs(v) < 1e-2 for v in rel.values()), (n, rel)
    # the finest level is within 0.2%
    n, q, qi = series[-1]
    assert abs(q["mass"] / tab["QoI-5"] - 1) < 2e-3
    assert abs(q["abs:B"] / tab["QoI-3"] - 1) < 2e-3
    assert abs(qi["abs:B"] / tab["QoI-4"] - 1) < 2e-3


def test_outflow_l15_is_twice_the_table(series):
    tab = _table()
    prev = 0.0
    for n, q, qi in series:
        r_t = q["out:S_1.5"] / tab["QoI-1 l=1.5"]
        r_i = qi["out:S_1.5"] / tab["QoI-2 l=1.5"]
        net = (q["out:S_1.5"] - q["in:S_1.5"]) / tab["QoI-1 l=1.5"]
        print(f"n={n}: gross outflow / table = {r_t:.4f} at T, {r_i:.4f} over [0, T]; net outflow / table {net:.4f}")
        assert 1.9 < r_t < 2.02 and 1.9 < r_i < 2.02, (n, r_t, r_i)
        assert abs(r_t / r_i - 1) < 5e-3  # the same factor at T and over time
        assert r_t > prev  # rising towards 2 under refinement
        prev = r_t
    # the net outflow does not match either
    n, q, qi = series[-1]
    assert abs((q["out:S_1.5"] - q["in:S_1.5"]) / tab["QoI-1 l=1.5"] - 1) > 0.5


def test_outflow_l25_far_from_the_table(series):
    tab = _table()
    for n, q, qi in series:
        assert q["out:S_2.5"] / tab["QoI-1 l=2.5"] > 300
        assert qi["out:S_2.5"] / tab["QoI-2 l=2.5"] > 300
