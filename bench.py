#!/usr/bin/env python3
"""Throughput of the explicit S_N transport step on one MI355X.

Workload (the headline line): the walled cavity on a 1300 x 1300 grid with
512 ordinates (8 Gauss-Legendre polar x 64 azimuths), minmod second order,
Heun, CFL 0.5 (5200 steps to T = 2.6); each FP32 psi buffer holds 3.5 GB,
far more than the 256 MB Infinity Cache. One step = both Heun stages with
their scalar-flux epilogues and QoI reductions over the whole grid. Inputs
are synthetic (the problem statement itself) and resident in HBM before
timing starts.

Prints one JSON line. `value` = cell-ordinate updates per second (one update
= one (cell, ordinate) advanced one full time step), timed over exactly
--steps steps with no per-launch instrumentation. `roofline` describes the
dominant kernel (Heun stage 2) against 8 TB/s, its average duration taken
with HIP events on the launch stream in a second, separately timed pass;
`step_roofline` is the whole step's algorithmic bytes over ms_per_step.
`cpu_baseline` times the FP64 oracle on a bounded sample of the same
workload on the host cores. Further keys time the 700^2 x 256 lattice, the
paper's tessellation quadrature and limiter, the Hohlraum, one GPU's share of
an ordinate split, the batched UQ workload and a compact serving sweep.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def source_digest():
    """SHA-256 over the kernel and ABI sources: ties a profile summary to the code it measured."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_2505_17284_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".h", ".cpp")))
    files.append(os.path.join(ROOT, "include", "snrt.h"))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, dtype, field="traffic_bytes_per_launch"):
    """HBM bytes per launch of the Heun stage-2 kernel (`field`
    traffic_bytes_per_launch_stage1: stage 1) on `workload` from the
    committed rocprofv3 counter summary, or None when the summary is missing
    or was taken on other sources. The summary is named for the grid and the
    ordinate count: stage_heun2_<workload without its stepper suffix>_<dtype>.md."""
    base = workload[: -len("_heun2")] if workload.endswith("_heun2") else workload
    path = os.path.join(PROFILES, f"stage_heun2_{base}_{dtype}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":", 1)[0].strip() in ("source_sha256", field):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256") != source_digest() or field not in fields:
        return None
    return float(fields[field])


# VALU issue peak without packed FP32 (which this build leaves off): one
# wave64 instruction per SIMD every 4 cycles, i.e. 16 lanes per cycle on each
# of the 1024 SIMDs (256 CUs x 4) at 2.4 GHz.
VALU_PEAK_LANE_OPS = 1024 * 16 * 2.4e9


def measured_valu():
    """SQ_INSTS_VALU per launch of the order-3 stage kernels (stage 1, stage 2)
    on the 700^2 x 256 lattice, FP32, from the committed counter summary, or
    None when it is missing or was taken on other sources."""
    path = os.path.join(PROFILES, "stage_venkat_lattice700_M256_f32.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":", 1)[0].strip() in ("source_sha256", "valu_insts_stage1",
                                                                  "valu_insts_stage2"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256") != source_digest() or "valu_insts_stage2" not in fields:
        return None
    return float(fields["valu_insts_stage1"]), float(fields["valu_insts_stage2"])


def algorithmic_bytes(problem, plan_info, kind):
    """Algorithmic HBM bytes of one stage launch over the whole grid.

    Per cell-ordinate: Heun stage 1 / Euler read psi and write psi (2 s);
    Heun stage 2 reads psi^(1) and psi^n and writes psi^(n+1) (3 s). Per cell:
    the incoming scalar flux (4 B), the outgoing one (4 B), the region id (1 B).
    Halo re-reads, partial-flux groups and padding are not algorithmic.
    """
    s = 2 if problem.psi_dtype == "bf16" else 4
    cells = problem.nx * problem.ny
    per_co = {0: 2 * s, 1: 2 * s, 2: 3 * s}[kind]
    return cells * problem.M * per_co + cells * 9


def cpu_baseline(problem, budget_s=12.0, share_M=64):
    """Time the oracle (as it stands) on whole Heun steps of the workload.

    Every oracle call copies the state and allocates its work arrays, so the
    rate comes from the difference of two calls (1 step, then 1 + s steps)
    on the same state. The one-thread figure takes a share of the ordinates
    (the cavity's grid with a share_M-ordinate product quadrature: the
    oracle's cost per cell-ordinate does not depend on M)."""
    import numpy as np

    import oracle
    from paper_2505_17284_amd import inputs as I

    oracle.build(force=False)
    threads = oracle.threads(0)

    def rate(p, budget):
        psi = np.zeros((p.M, p.ny, p.nx))
        t0 = time.perf_counter()
        psi, _ = oracle.advance(p, psi, 1)
        one = time.perf_counter() - t0
        steps = max(1, min(50, int(budget / max(one, 1e-6))))
        t0 = time.perf_counter()
        psi1, _ = oracle.advance(p, psi, 1)
        t1 = time.perf_counter() - t0
        del psi1
        t0 = time.perf_counter()
        psi2, _ = oracle.advance(p, psi, 1 + steps)
        t2 = time.perf_counter() - t0
        del psi, psi2
        return p.cell_ordinates * steps / max(t2 - t1, 1e-9), steps, t2 - t1

    ups, steps, secs = rate(problem, budget_s)
    share = problem.replace(quad=I.quadrature_for(share_M), name=f"{problem.name}_M{share_M}")
    oracle.threads(1)
    try:
        ups1, steps1, secs1 = rate(share, 4.0)
    finally:
        oracle.threads(threads)
    return {"value": ups, "unit": "cell-ordinate updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} Heun steps of the {problem.nx}x{problem.ny}x{problem.M} {problem.meta.get('kind', '')} "
                      f"(FP64, {threads} OpenMP threads, {secs:.1f} s net of one call's set-up)",
            "value_1_thread": ups1,
            "sample_1_thread": f"{steps1} Heun step(s) of the {share.nx}x{share.ny} grid with {share_M} of the "
                               f"ordinates on one thread ({secs1:.1f} s)"}


def time_workload(p, workload, steps, warmup=3, kernel_steps=None):
    """Heun steps of a full-size workload: wall-clock time of exactly `steps`
    steps with no per-launch instrumentation (ms_per_step, updates/s, the
    step's algorithmic rate), then the two stage kernels' average durations
    from HIP events on the launch stream over a second pass of
    `kernel_steps` steps."""
    import torch

    from paper_2505_17284_amd import solver

    kernel_steps = kernel_steps or steps
    print(f"[bench] {workload}: {p.name} {steps} steps", file=sys.stderr, flush=True)
    plan = solver.Plan(p, device="cuda:0")
    try:
        plan.run(warmup, unbounded=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run(steps, unbounded=True)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        plan.set_timing(True)
        plan.run(kernel_steps, unbounded=True)
        torch.cuda.synchronize()
        ms, counts = plan.kernel_ms()
        plan.set_timing(False)
        info = plan.info
    finally:
        plan.close()
    s2 = ms[2] / max(counts[2], 1)
    s1 = ms[1] / max(counts[1], 1)
    b2 = algorithmic_bytes(p, info, 2)
    b1 = algorithmic_bytes(p, info, 1)
    step_gbs = (b1 + b2) / (secs / steps) / 1e9
    return {"workload": workload, "steps": steps, "ms_per_step": secs * 1e3 / steps,
            "updates_per_s": p.cell_ordinates * steps / secs, "stage2_kernel_ms": s2,
            "stage2_achieved_GBs": b2 / (s2 * 1e-3) / 1e9, "stage2_frac": b2 / (s2 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "stage1_kernel_ms": s1, "stage1_achieved_GBs": b1 / (s1 * 1e-3) / 1e9,
            "stage1_frac": b1 / (s1 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "kernel_steps": kernel_steps, "step_algorithmic_GBs": step_gbs, "step_frac": step_gbs / HBM_PEAK_GBS,
            "step_algorithmic_bytes": b1 + b2, "stage1_bytes": b1, "stage2_bytes": b2,
            "ordinates_per_group": [info["group_size"], info["group_size_average"]], "info": info}


def time_lattice(steps, dtype, warmup=3):
    """The 700^2 lattice with 256 ordinates (minmod, Heun): 0.5 GB per FP32
    psi buffer, partly held by the 256 MB Infinity Cache."""
    from paper_2505_17284_amd import inputs as I

    return time_workload(I.config(2).replace(psi_dtype=dtype), "lattice700_M256_heun2", steps, warmup)


def time_tessellation(steps, dtype, N=22, warmup=2):
    """The lattice at 700^2 with the paper's tessellation quadrature at its
    finest N = 22 (M = 4 N^2 = 1936 ordinates, 3.8 GB per FP32 psi buffer)."""
    from paper_2505_17284_amd import inputs as I

    p = I.lattice(700, order=2, stepper=I.HEUN, quad=I.tessellation_quadrature(N), psi_dtype=dtype,
                  name=f"lattice700_tess{N}")
    return time_workload(p, f"lattice700_tess{N}_M{4 * N * N}_heun2", steps, warmup)


def time_hohlraum(steps, dtype, n=1300, M=256, warmup=2):
    """The Hohlraum (layout Sec. 3.2.1, QoIs Sec. 3.2.2) at n^2 cells with every QoI on: the four
    probes' windows (QoI-1) and the fluence behind QoI-3 to QoI-6, timed
    against the same solve without them (same launch shape)."""
    import torch

    from paper_2505_17284_amd import hohlraum
    from paper_2505_17284_amd import inputs as I
    from paper_2505_17284_amd import solver

    p = I.hohlraum(n, M, psi_dtype=dtype)
    out = {"workload": f"hohlraum{n}_M{M}_heun2", "steps": steps}
    qois = {"probes": hohlraum.probe_cells(p), "fluence": True}
    # both solves at the launch shape the one with QoIs takes by default
    info = solver.plan_info(p, **qois)
    shape = {k: info[k] for k in ("rows_per_wave", "waves_per_group", "group_size", "group_size_average")}
    out["shape"] = shape
    for label, kw in (("plain", {}), ("with_qois", qois)):
        print(f"[bench] hohlraum {label}: {p.name} {steps} steps", file=sys.stderr, flush=True)
        plan = solver.Plan(p, device="cuda:0", **shape, **kw)
        try:
            plan.run(warmup, unbounded=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.run(steps, unbounded=True)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            if kw:
                out["green_band_A_G"] = hohlraum.green_band_qois(plan)["A_G"]
        finally:
            plan.close()
        out[f"ms_per_step_{label}"] = secs * 1e3 / steps
        out[f"updates_per_s_{label}"] = p.cell_ordinates * steps / secs
    out["qoi_overhead"] = out["ms_per_step_with_qois"] / out["ms_per_step_plain"] - 1.0
    return out


def time_venkat(steps, dtype, warmup=2):
    """The benchmark lattice (700^2, 256 ordinates, Heun) with the paper's own
    limiter: the Green-Gauss gradient with the Venkatakrishnan limiter (order 3)."""
    from paper_2505_17284_amd import inputs as I

    p = I.config(2).replace(order=3, psi_dtype=dtype, name="lattice700_M256_venkat")
    out = time_workload(p, "lattice700_M256_heun_venkat", steps, warmup)
    valu = measured_valu() if dtype == "f32" else None
    if valu is not None:
        # bound by its arithmetic: VALU lane-instructions per second against the issue peak
        achieved = valu[1] * 64 / (out["stage2_kernel_ms"] * 1e-3)
        out["alu"] = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_LANE_OPS,
                      "unit": "VALU lane-instructions/s (SQ_INSTS_VALU x 64 / kernel time)",
                      "frac": achieved / VALU_PEAK_LANE_OPS, "kernel": "sn_stage_kernel<3, kAverage>",
                      "stage1_frac": valu[0] * 64 / (out["stage1_kernel_ms"] * 1e-3) / VALU_PEAK_LANE_OPS}
    return out


def stream_ceiling(mib, reps=5):
    """What plain streaming kernels reach on this GPU: torch's elementwise
    add (two reads, one write: the mix of Heun's averaging stage) and a
    device copy (one read, one write: the update stage), mib MiB per array,
    best of `reps` launches timed with events."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    out = {"bytes_per_array": n * 4}
    for label, fn, arrays in (("add", lambda: torch.add(a, b, out=c), 3), ("copy", lambda: c.copy_(a), 2)):
        fn()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[f"{label}_GBs"] = arrays * n * 4 / (best * 1e-3) / 1e9
    del a, b, c
    torch.cuda.synchronize()
    return out


def time_shard(steps, dtype, shards=8, warmup=3):
    """One GPU's share of the full-size cavity split by ordinates over
    `shards` GPUs: 1300^2 cells with 512 / shards ordinates (a product
    quadrature of that size, which costs the same as a subset of the 512).
    Each stage of a split solve ends with an all-reduce of the nx ny FP32
    scalar-flux partial; its size is reported beside the stage times."""
    from paper_2505_17284_amd import inputs as I

    M = 512 // shards
    p = I.cavity(1300, M, psi_dtype=dtype, name=f"cavity1300_M{M}")
    out = time_workload(p, f"cavity1300_M{M}_heun2 (1/{shards} of 512 ordinates)", steps, warmup)
    out["phi_allreduce_bytes_per_stage"] = p.nx * p.ny * 4
    return out


HEADLINE = "cavity1300_M512_heun2"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--kernel-steps", type=int, default=20,
                    help="steps of the second, event-timed pass that gives the per-kernel averages")
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--group", type=int, default=0, help="ordinates per workgroup, both stages (0: default)")
    ap.add_argument("--group-avg", type=int, default=0, help="ordinates per workgroup of the averaging stage")
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--uq", type=int, default=256,
                    help="instances of the batched UQ workload (0 skips it)")
    ap.add_argument("--serving-requests", type=int, default=32,
                    help="requests per rate of the serving sweep (0 skips it)")
    ap.add_argument("--serving-loads", default="0.5,0.9,1.1",
                    help="arrival rates of the serving sweep as fractions of the one-at-a-time capacity")
    ap.add_argument("--serving-policies", default="deadline",
                    help="continuous-batching policies compared with one solve at a time")
    ap.add_argument("--lattice-steps", type=int, default=100,
                    help="Heun steps timed on the 700^2 x 256 lattice (0 skips it)")
    ap.add_argument("--tess-steps", type=int, default=10,
                    help="Heun steps timed on the 700^2 lattice with the tessellation quadrature, "
                         "N = 22 (1936 ordinates; 0 skips it)")
    ap.add_argument("--venkat-steps", type=int, default=40,
                    help="Heun steps timed on the benchmark lattice with the Venkatakrishnan limiter "
                         "(order 3; 0 skips it)")
    ap.add_argument("--hohlraum-steps", type=int, default=20,
                    help="Heun steps timed on the 1300^2 x 256 Hohlraum with and without its probes and "
                         "fluence (0 skips it)")
    ap.add_argument("--shard-steps", type=int, default=40,
                    help="Heun steps timed on one GPU's share of an 8-way ordinate split of the cavity, "
                         "1300^2 x 64 ordinates (0 skips it)")
    ap.add_argument("--other-dtype", action="store_true",
                    help="also time the headline workload with the other psi storage type")
    ap.add_argument("--stream-mib", type=int, default=1024,
                    help="MiB per array of the streaming-ceiling measurement (0 skips it)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after timing, run one device-to-device copy of this many MiB "
                         "(reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU angular split is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2505_17284_amd import inputs as I
    from paper_2505_17284_amd import solver

    problem = I.config(3).replace(psi_dtype=args.dtype)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    plan = solver.Plan(problem, group_size=args.group, rows_per_wave=args.rows, waves_per_group=args.waves,
                       device="cuda:0", group_size_average=args.group_avg)
    info = plan.info
    print(f"[bench] plan: {info}", file=sys.stderr, flush=True)
    plan.run(args.warmup, unbounded=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(args.steps, unbounded=True)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    print(f"[bench] timed {args.steps} steps in {secs:.4f} s", file=sys.stderr, flush=True)
    # second pass: per-launch HIP events on the launch stream
    plan.set_timing(True)
    plan.run(args.kernel_steps, unbounded=True)
    torch.cuda.synchronize()
    ms, counts = plan.kernel_ms()
    plan.set_timing(False)
    plan.close()
    print(f"[bench] kernel pass: {args.kernel_steps} steps, kernel ms {ms} counts {counts}",
          file=sys.stderr, flush=True)

    ups = problem.cell_ordinates * args.steps / secs
    kind = 2  # Heun stage 2 dominates (3 psi accesses per cell-ordinate)
    avg_ms = ms[kind] / max(counts[kind], 1)
    bytes_launch = algorithmic_bytes(problem, info, kind)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    stage1_bytes = algorithmic_bytes(problem, info, 1)
    stage1_ms = ms[1] / max(counts[1], 1)
    stage1_gbs = stage1_bytes / (stage1_ms * 1e-3) / 1e9
    step_bytes = stage1_bytes + bytes_launch
    step_gbs = step_bytes / (secs / args.steps) / 1e9
    traffic = traffic1 = None
    default_shape = not (args.group or args.group_avg or args.rows or args.waves)
    if default_shape:
        traffic = measured_traffic(HEADLINE, args.dtype)
        traffic1 = measured_traffic(HEADLINE, args.dtype, "traffic_bytes_per_launch_stage1")
    line = {
        "metric": "cell-ordinate updates/s",
        "value": ups,
        "unit": "cell-ordinate updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": HEADLINE, "nx": problem.nx, "ny": problem.ny,
                   "ordinates": problem.M, "order": problem.order, "stepper": "heun",
                   "cfl": problem.cfl, "n_steps_to_T": info["n_steps"], "psi_storage": args.dtype,
                   "group_size": info["group_size"], "group_size_average": info["group_size_average"],
                   "rows_per_wave": info["rows_per_wave"],
                   "waves_per_group": info["waves_per_group"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "sn_stage_kernel<2, kAverage> (Heun stage 2)",
                     "kernel_avg_ms": avg_ms, "kernel_launches_timed": counts[kind],
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, "
                                     "calibrated on a device copy)",
                     "traffic_over_algorithmic": None if traffic is None else traffic / bytes_launch},
        "step_roofline": {"bound": "hbm", "achieved": step_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": step_gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_step": step_bytes,
                          "note": "both stages' algorithmic bytes over the wall-clock ms_per_step "
                                  "(finalize launches and gaps included)"},
        "stage1": {"kernel_avg_ms": stage1_ms, "achieved_GBs": stage1_gbs, "frac": stage1_gbs / HBM_PEAK_GBS,
                   "algorithmic_bytes_per_launch": stage1_bytes, "traffic": traffic1,
                   "traffic_over_algorithmic": None if traffic1 is None else traffic1 / stage1_bytes},
        "roofline_updates_per_s": HBM_PEAK_GBS * 1e9 / (step_bytes / problem.cell_ordinates),
    }
    if args.stream_mib:
        ceil = stream_ceiling(args.stream_mib)
        line["stream_ceiling"] = ceil
        line["roofline"]["frac_of_stream_ceiling"] = achieved / ceil["add_GBs"]
        line["stage1"]["frac_of_copy_ceiling"] = stage1_gbs / ceil["copy_GBs"]
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = n
        del src, dst
    if args.other_dtype:
        other = "bf16" if args.dtype == "f32" else "f32"
        line[f"cavity_{other}"] = time_workload(I.config(3).replace(psi_dtype=other), HEADLINE + f"_{other}",
                                                min(args.steps, 40), 3, args.kernel_steps)
        line[f"cavity_{other}"].pop("info")
    if args.lattice_steps:
        line["lattice700"] = time_lattice(args.lattice_steps, args.dtype)
        line["lattice700"].pop("info")
    if args.tess_steps:
        line["tessellation"] = time_tessellation(args.tess_steps, args.dtype)
        line["tessellation"].pop("info")
    if args.venkat_steps:
        line["venkat"] = time_venkat(args.venkat_steps, args.dtype)
        line["venkat"].pop("info", None)
    if args.hohlraum_steps:
        line["hohlraum"] = time_hohlraum(args.hohlraum_steps, args.dtype)
    if args.shard_steps:
        line["shard_share"] = time_shard(args.shard_steps, args.dtype)
        line["shard_share"].pop("info")
    from paper_2505_17284_amd import serve

    if args.uq:
        print(f"[bench] batched UQ: {args.uq} lattice draws", file=sys.stderr, flush=True)
        line["batched_uq"] = serve.uq(args.uq, verbose=True, compare_tuned=True)
    if args.serving_requests:
        loads = tuple(float(x) for x in args.serving_loads.split(","))
        print(f"[bench] serving: {args.serving_requests} requests at loads {loads}", file=sys.stderr, flush=True)
        line["serving"] = serve.sweep(args.serving_requests, rates=loads, verbose=False,
                                      policies=tuple(args.serving_policies.split(",")))
    if not args.no_cpu:
        print("[bench] cpu baseline (FP64 oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(problem)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
