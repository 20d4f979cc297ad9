"""Write oracle QoIs of full benchmark solves to tests/golden/.

Calls only the FP64 oracle (oracle/) and the seeded problem generators; no
value here comes from the HIP path.

    python tests/golden/make_oracle_goldens.py lattice700   # ~10 min on 8 cores
    python tests/golden/make_oracle_goldens.py hohlraum260  # ~2 min on 8 cores
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
from paper_2505_17284_amd import inputs as I  # noqa: E402

CASES = {
    "lattice700": ("oracle_lattice700_M256_heun2.json", lambda: I.config(2)),
    "lattice70": ("oracle_lattice70_M32_euler1.json", lambda: I.config(1)),
    "hohlraum260": ("oracle_hohlraum260_M256_heun2.json", lambda: I.hohlraum(260, 256)),
}


def main(names):
    oracle.build(force=False)
    for name in names:
        fname, make = CASES[name]
        p = make()
        t0 = time.time()
        r = oracle.solve(p)
        out = dict(
            problem=p.name, nx=p.nx, ny=p.ny, M=p.M, order=p.order, stepper=p.stepper,
            nt=r["nt"], dt=r["dt"], t=r["t"],
            qoi=dict(zip(r["names"], map(float, r["qoi"]))),
            qoi_int=dict(zip(r["names"], map(float, r["qoi_int"]))),
            oracle_seconds=time.time() - t0, oracle_threads=oracle.threads(0),
            host=platform.processor() or platform.machine(),
            writer="tests/golden/make_oracle_goldens.py (FP64 oracle only)",
        )
        with open(os.path.join(HERE, fname), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "done in", round(out["oracle_seconds"], 1), "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
