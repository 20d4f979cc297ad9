"""Write oracle QoIs of full benchmark solves to tests/golden/.

Calls only the FP64 oracle (oracle/) and the seeded problem generators; no
value here comes from the HIP path.

    python tests/golden/make_oracle_goldens.py lattice700   # ~10 min on 8 cores
    python tests/golden/make_oracle_goldens.py hohlraum260  # ~2 min on 8 cores
    python tests/golden/make_oracle_goldens.py uq8          # ~25 min on 8 cores
    python tests/golden/make_oracle_goldens.py cavity1300   # ~2 h on 8 cores, 3.5 GB

``uq8`` stores eight DP-2 lattice draws (one list) whose seeds span every
grid side {140, 280, 420, 560} and ordinate count {64, 128, 256}.
``cavity1300`` is the walled cavity at its full grid and length (1300^2,
5200 Heun steps) with 64 of the 512 ordinates' worth of work: the 4 x 16
product quadrature.

Hohlraum cases also store the green-band QoI-3 to QoI-6 of the oracle's
fluence and the QoI-1 probe windows (oracle/hohlraum_qoi.py).
"""

import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import hohlraum_qoi  # noqa: E402
from paper_2505_17284_amd import inputs as I  # noqa: E402

CASES = {
    "lattice700": ("oracle_lattice700_M256_heun2.json", lambda: I.config(2)),
    "lattice70": ("oracle_lattice70_M32_euler1.json", lambda: I.config(1)),
    "hohlraum260": ("oracle_hohlraum260_M256_heun2.json", lambda: I.hohlraum(260, 256)),
    "cavity1300": ("oracle_cavity1300_M64_heun2.json",
                   lambda: I.cavity(1300, 64, name="cavity1300_M64_heun2")),
}

# DP-2 draws: (seed, n, M) = (10, 560, 256), (0, 560, 128), (2, 560, 64),
# (4, 420, 256), (16, 420, 128), (9, 280, 256), (24, 280, 64), (35, 140, 128).
UQ_SEEDS = (10, 0, 2, 4, 16, 9, 24, 35)
UQ_FILE = "oracle_uq8_heun2.json"


def _record(p, r, t0):
    return dict(
        problem=p.name, nx=p.nx, ny=p.ny, M=p.M, order=p.order, stepper=p.stepper,
        nt=r["nt"], dt=r["dt"], t=r["t"],
        qoi=dict(zip(r["names"], map(float, r["qoi"]))),
        qoi_int=dict(zip(r["names"], map(float, r["qoi_int"]))),
        oracle_seconds=time.time() - t0, oracle_threads=oracle.threads(0),
        host=platform.processor() or platform.machine(),
        writer="tests/golden/make_oracle_goldens.py (FP64 oracle only)",
    )


def uq8():
    runs = []
    for seed in UQ_SEEDS:
        p = I.uq_instance(seed)
        t0 = time.time()
        rec = _record(p, oracle.solve(p), t0)
        rec["seed"] = seed
        runs.append(rec)
        print(p.name, "done in", round(rec["oracle_seconds"], 1), "s", flush=True)
    with open(os.path.join(HERE, UQ_FILE), "w") as f:
        json.dump({"seeds": list(UQ_SEEDS), "runs": runs}, f, indent=1)


def main(names):
    oracle.build(force=False)
    for name in names:
        if name == "uq8":
            uq8()
            continue
        fname, make = CASES[name]
        p = make()
        t0 = time.time()
        hohl = p.meta.get("kind") == "hohlraum"
        r = oracle.solve(p, fluence=hohl, probes=hohlraum_qoi.probe_cells(p) if hohl else None)
        out = _record(p, r, t0)
        if hohl:
            band = hohlraum_qoi.qois(p, r["fluence"])
            out["green_band"] = {k: float(band[k]) for k in ("A_G", "V_G", "A_L", "V_L", "length")}
            out["green_band"]["A"] = [float(a) for a in band["A"]]
            out["probes"] = r["probes"].tolist()  # [window][probe][phi, J_x, J_y]
        with open(os.path.join(HERE, fname), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "done in", round(out["oracle_seconds"], 1), "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES) + ["uq8"])
