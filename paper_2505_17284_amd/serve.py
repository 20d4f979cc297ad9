"""Request loops over the batched S_N solver: continuous batching vs one solve at a time.

Continuous batching (``serve``): requests arrive on a wall clock (Poisson
arrivals from ``inputs.serving_requests``); a request is admitted as soon as a
slot of the batch for its storage type and the shared HBM budget allow, its
state stays on the device, and every window of K steps advances all admitted
unfinished requests together (one persistent launch per stage, replayed from a
captured hipGraph while the set is unchanged). Finished requests return their
QoIs to the host and free their slot and memory at once.

The plain path (``serve_fifo``) solves one request at a time in arrival order
with the single-plan API.

Latency = time from a request's arrival to its QoIs on the host.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import batch as B
from . import inputs as I
from . import solver


def _sync():
    import torch

    torch.cuda.synchronize()


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else float("nan")


def step_cost(p) -> float:
    """Bytes one step of a problem moves (cells x ordinates x bytes per stored psi)."""
    return float(p.cell_ordinates) * (2.0 if p.psi_dtype == "bf16" else 4.0)


def work_quotas(costs: dict, k: int) -> dict:
    """Steps per run so that every admitted problem gets about the same GPU
    time per run: the cheapest takes k steps, a problem c times as expensive
    k / c (at least 1)."""
    if not costs:
        return {}
    cmin = min(costs.values())
    return {key: max(1, min(k, int(round(k * cmin / c)))) for key, c in costs.items()}


def arrival_quotas(order: list, costs: dict, k: int, backfill: float = 0.25, min_work: float = 2e9,
                   k_max: int | None = None) -> dict:
    """Steps per run that keep arrival order: the oldest admitted request takes
    k steps (more, up to k_max, while that is less than min_work bytes of psi
    steps, so that a run is never mostly overhead); later ones, oldest first,
    fill in until the run holds max(k cost(oldest) (1 + backfill), min_work)
    bytes of psi steps (so that short requests ride along with a long one and
    many short ones fill the GPU together); a request that no longer fits is
    paused for the run."""
    if not order:
        return {}
    head = order[0]
    if k_max is not None and k_max > k:
        k = max(k, min(k_max, int(min_work // costs[head])))
    target = max(k * costs[head] * (1.0 + backfill), min_work)
    used = 0.0
    out = {}
    for key in order:
        c = costs[key]
        steps = k if key == head else min(k, int((target - used) // c))
        if steps <= 0:
            out[key] = B.PAUSED
            continue
        out[key] = steps
        used += steps * c
    return out


def response_ratio_order(keys, wait_s: dict, rem_s: dict, tiebreak: dict) -> list:
    """keys by highest response ratio first, (wait + remaining) / remaining
    (both in seconds; ties by `tiebreak`, e.g. arrival order): a short request
    outranks a long one that has waited as long, and a long one outranks short
    ones once it has waited long enough relative to its own remaining time."""
    return sorted(keys, key=lambda k: (-(wait_s[k] + rem_s[k]) / rem_s[k], tiebreak[k]))


def deadline_order(keys, arrival_s: dict, service_s: dict, tiebreak: dict, slowdown: float) -> list:
    """keys by earliest deadline first, deadline = arrival + slowdown x the
    request's whole service time alone (ties by `tiebreak`): a short request
    gets an early deadline and overtakes long ones, but every request's
    deadline comes up at a fixed multiple of its own service time, which
    bounds how long a long request waits behind a stream of short ones."""
    return sorted(keys, key=lambda k: (arrival_s[k] + slowdown * service_s[k], tiebreak[k]))


def serve(requests, hbm_budget_bytes: int, max_instances: int = 64, steps_per_run: int = 32,
          rows_per_wave: int = 2, waves_per_group: int = 4, policy: str = "deadline", verbose: bool = False,
          batch_factory=None, max_steps_per_run: int = 256, run_work: float = 2e10, service_rate: float = 8e11,
          slowdown: float = 4.0):
    """Continuous batching over `requests` = [(arrival_s, Problem)], Heun + minmod.

    policy "srpt": the admitted request with the least remaining work (psi
    steps x bytes per step) takes full runs and the others fill in by the same
    rule, so short requests overtake long ones that are already running (the
    GPU is shared by preemption at run boundaries; each request still runs at
    the full speed of its own kernels); "hrrn": the same with the highest
    response ratio (time since arrival + remaining time) / remaining time
    first, re-ranked every run, the remaining time estimated from the rate
    measured so far (service_rate psi-step bytes per second until then):
    short requests still overtake, but a long one's ratio grows while it
    waits, which bounds its delay; "deadline" (the default): the same with
    the earliest deadline first, deadline = arrival + slowdown x the
    request's whole service time at the measured rate (short requests still
    overtake, and no request's slowdown grows without bound); "arrival": the
    same with the oldest
    request first, so no request is slowed much by later arrivals; "work": per-run step quotas share the GPU by work (short
    requests finish fast, long ones are slowed down); "steps": every admitted
    request takes steps_per_run steps per run. With "arrival" a run holds at
    least run_work bytes of psi steps (up to max_steps_per_run steps of the
    oldest request), so that runs of short requests are not mostly overhead.
    Returns per-request records and totals. batch_factory (default
    batch.Batch) builds one batch per storage type; the host-only tests pass a
    stand-in that models the device."""
    dtypes = sorted({p.psi_dtype for _, p in requests})
    make = batch_factory or B.Batch
    k_max = max(steps_per_run, max_steps_per_run if policy in ("arrival", "srpt", "deadline") else steps_per_run)
    n_steps = [solver.plan_info(p)["n_steps"] for _, p in requests]
    batches = {d: make(order=2, stepper=I.HEUN, psi_dtype=d, max_instances=max_instances,
                       steps_per_run=k_max, rows_per_wave=rows_per_wave,
                       waves_per_group=waves_per_group) for d in dtypes}
    fps = [B.footprint(p, rows_per_wave, waves_per_group) for _, p in requests]
    for i, f in enumerate(fps):
        if f > hbm_budget_bytes:
            raise ValueError(f"request {i} needs {f} bytes, more than the whole budget")
    used = 0
    peak = 0
    queue: list[int] = []
    slot_of: dict[tuple, int] = {}
    rec = [dict(arrival=a, name=p.name, n=p.nx, M=p.M, dtype=p.psi_dtype, cell_ord_steps=0,
                admitted=None, done=None) for a, p in requests]
    nxt = 0
    finished = 0
    changed = False
    t0 = time.perf_counter()
    windows = 0
    busy_s, work_done = 0.0, 0.0  # measured service rate (hrrn)
    try:
        while finished < len(requests):
            now = time.perf_counter() - t0
            while nxt < len(requests) and requests[nxt][0] <= now:
                queue.append(nxt)
                nxt += 1
            # FIFO admission, no overtaking: the head waits for budget or a slot
            while queue:
                i = queue[0]
                p = requests[i][1]
                b = batches[p.psi_dtype]
                if used + fps[i] > hbm_budget_bytes or len(b.plans) >= max_instances:
                    break
                queue.pop(0)
                s = b.admit(p)
                slot_of[(p.psi_dtype, s)] = i
                used += fps[i]
                peak = max(peak, used)
                rec[i]["admitted"] = time.perf_counter() - t0
                changed = True
            if changed:
                costs = {key: step_cost(requests[i][1]) for key, i in slot_of.items()}
                if policy == "work":
                    quotas = work_quotas(costs, steps_per_run)
                elif policy == "arrival":
                    order = sorted(slot_of, key=lambda key: slot_of[key])  # request index = arrival order
                    quotas = arrival_quotas(order, costs, steps_per_run, min_work=run_work, k_max=k_max)
                elif policy == "srpt":
                    rem = {key: costs[key] * (n_steps[i] - batches[key[0]].status(key[1])[1])
                           for key, i in slot_of.items()}
                    order = sorted(slot_of, key=lambda key: (rem[key], slot_of[key]))
                    quotas = arrival_quotas(order, costs, steps_per_run, backfill=0.1, min_work=run_work, k_max=k_max)
                elif policy == "deadline":
                    rate = work_done / busy_s if busy_s > 0 and work_done > 0 else service_rate
                    service_s = {key: costs[key] * n_steps[i] / rate for key, i in slot_of.items()}
                    arrival_s = {key: requests[i][0] for key, i in slot_of.items()}
                    order = deadline_order(list(slot_of), arrival_s, service_s, slot_of, slowdown)
                    quotas = arrival_quotas(order, costs, steps_per_run, backfill=0.1, min_work=run_work, k_max=k_max)
                elif policy == "hrrn":
                    rate = work_done / busy_s if busy_s > 0 and work_done > 0 else service_rate
                    now = time.perf_counter() - t0
                    rem_s = {key: max(costs[key] * (n_steps[i] - batches[key[0]].status(key[1])[1]) / rate, 1e-6)
                             for key, i in slot_of.items()}
                    wait_s = {key: now - requests[i][0] for key, i in slot_of.items()}
                    order = response_ratio_order(list(slot_of), wait_s, rem_s, slot_of)
                    quotas = arrival_quotas(order, costs, steps_per_run, backfill=0.1, min_work=run_work, k_max=k_max)
                else:
                    quotas = {key: steps_per_run for key in costs}
                for (d, s), q in quotas.items():
                    batches[d].set_steps(s, q)
                changed = False
            active = [b for b in batches.values() if b.unfinished()]
            if not active:
                if nxt < len(requests):
                    time.sleep(max(0.0, requests[nxt][0] - (time.perf_counter() - t0)))
                continue
            if policy in ("hrrn", "deadline"):
                before = {key: batches[key[0]].status(key[1])[1] for key in slot_of}
                tw = time.perf_counter()
            for b in active:
                b.run()
            windows += 1
            for b in active:
                b.synchronize()
            if policy in ("hrrn", "deadline"):
                busy_s += time.perf_counter() - tw
                work_done += sum(costs[key] * (batches[key[0]].status(key[1])[1] - st) for key, st in before.items())
                changed = changed or policy == "hrrn"  # ratios move with time: re-rank every run
            for d, b in batches.items():
                for s in b.done_slots():
                    i = slot_of.pop((d, s))
                    r = b.result(s, allow_nonfinite=True)
                    rec[i]["done"] = time.perf_counter() - t0
                    rec[i]["nonfinite"] = r["nonfinite"]
                    rec[i]["latency"] = rec[i]["done"] - rec[i]["arrival"]
                    rec[i]["nt"] = r["nt"]
                    rec[i]["qoi_int"] = r["qoi_int"]
                    rec[i]["cell_ord_steps"] = requests[i][1].cell_ordinates * r["nt"]
                    b.retire(s)
                    used -= fps[i]
                    finished += 1
                    changed = True
                    if verbose:
                        print(f"[serve] {rec[i]['name']} latency {rec[i]['latency']:.3f} s", file=sys.stderr,
                              flush=True)
    finally:
        for b in batches.values():
            b.close()
    wall = time.perf_counter() - t0
    return rec, dict(wall_s=wall, windows=windows, peak_bytes=peak)


def serve_fifo(requests, verbose: bool = False, rows_per_wave: int = 2, waves_per_group: int = 4):
    """One request at a time, in arrival order, through the single-plan path."""
    rec = []
    t0 = time.perf_counter()
    for a, p in requests:
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        start = time.perf_counter() - t0
        plan = solver.Plan(p, rows_per_wave=rows_per_wave, waves_per_group=waves_per_group)
        try:
            plan.run()
            r = plan.qoi(allow_nonfinite=True)
            r["nt"] = plan.n_steps
        finally:
            plan.close()
        done = time.perf_counter() - t0
        rec.append(dict(arrival=a, name=p.name, n=p.nx, M=p.M, dtype=p.psi_dtype, start=start, done=done,
                        latency=done - a, service=done - start, nt=r["nt"], qoi_int=r["qoi_int"],
                        nonfinite=r["nonfinite"],
                        cell_ord_steps=p.cell_ordinates * r["nt"]))
        if verbose:
            print(f"[fifo] {p.name} service {done - start:.3f} s latency {done - a:.3f} s", file=sys.stderr,
                  flush=True)
    return rec, dict(wall_s=time.perf_counter() - t0)


def summarize(rec, totals, alone_service=None):
    lat = [r["latency"] for r in rec]
    first = min(r["arrival"] for r in rec)
    last = max(r["done"] for r in rec)
    out = dict(requests=len(rec), nonfinite=sum(1 for r in rec if r.get("nonfinite")), p50_latency_s=percentile(lat, 50), p99_latency_s=percentile(lat, 99),
               mean_latency_s=float(np.mean(lat)), solves_per_s=len(rec) / max(last - first, 1e-9),
               updates_per_s=sum(r["cell_ord_steps"] for r in rec) / max(last - first, 1e-9), **totals)
    if alone_service is not None:
        slow = [r["latency"] / max(alone_service[r["name"]], 1e-9) for r in rec]
        out["p99_slowdown"] = percentile(slow, 99)
        out["p50_slowdown"] = percentile(slow, 50)
    return out


def same_results(rec_a, rec_b, rtol: float = 1e-5):
    """Largest relative difference of any integrated QoI between two runs of the same requests."""
    worst = 0.0
    for a, b in zip(rec_a, rec_b):
        assert a["name"] == b["name"]
        for k, va in a["qoi_int"].items():
            vb = b["qoi_int"][k]
            scale = max(abs(va), abs(vb), 1e-300)
            worst = max(worst, abs(va - vb) / scale)
    return worst


def uq(n_instances: int = 256, seed0: int = 0, steps_per_run: int = 16, compare_alone: bool = True,
       psi_dtype: str = "f32", verbose: bool = False, tune: bool = False, compare_default: bool = False,
       direct_per_cu: int = 4, compare_tuned: bool = False):
    """The batched UQ workload: DP-2 lattice draws, all admitted at once, run to T.
    tune: admit every draw with the ordinate groups `solver.autotune` measures
    for its (grid, ordinates) class (tuning time reported apart, not in
    wall_s); the one-at-a-time comparison then uses the same groups, so that
    speedup_vs_alone is the batching's alone. compare_default: also run the
    batch with the library's default groups (speedup_vs_default_shapes).
    compare_tuned (with tune False): also run the batch with the autotuned
    groups (tuned_wall_s, tuned_tune_s, speedup_tuned_vs_default).
    direct_per_cu: plans with at least this many workgroups per compute unit
    take launches of their own (the library's default is 2; with many small
    plans at once, as here, 4 measured faster: 15.3 vs 16.4 s)."""
    probs = [I.uq_instance(seed0 + s, psi_dtype=psi_dtype) for s in range(n_instances)]
    shapes = [dict() for _ in probs]
    tune_s = 0.0
    if tune:
        t0 = time.perf_counter()
        for p, sh in zip(probs, shapes):
            t = solver.autotune(p)
            sh.update(group_size=t["group_size"], group_size_average=t["group_size_average"])
        _sync()
        tune_s = time.perf_counter() - t0
    work = 0
    for p in probs:
        nt = solver.plan_info(p)["n_steps"]
        work += p.cell_ordinates * nt
    _sync()
    t0 = time.perf_counter()
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    b = B.Batch(order=2, stepper=I.HEUN, psi_dtype=psi_dtype, max_instances=n_instances,
                steps_per_run=steps_per_run, direct_min_workgroups=direct_per_cu * cus)
    try:
        slots = [b.admit(p, **sh) for p, sh in zip(probs, shapes)]
        t_admit = time.perf_counter() - t0
        while b.unfinished():
            b.run()
        res = [b.result(s) for s in slots]
        _sync()
        secs = time.perf_counter() - t0
        info = b.info()
        peak = info["bytes_admitted"]
    finally:
        b.close()
    out = dict(instances=n_instances, tuned=tune, tune_s=tune_s, wall_s=secs, admit_s=t_admit,
               solves_per_s=n_instances / secs,
               updates_per_s=work / secs, cell_ord_steps=work, peak_bytes=peak,
               graph_replays=info["graph_replays"], launches=info["launches"])
    if compare_default and tune:
        d = uq(n_instances, seed0, steps_per_run, compare_alone=False, psi_dtype=psi_dtype, tune=False,
               direct_per_cu=direct_per_cu)
        out["default_shapes_wall_s"] = d["wall_s"]
        out["speedup_vs_default_shapes"] = d["wall_s"] / secs
    if compare_tuned and not tune:
        t = uq(n_instances, seed0, steps_per_run, compare_alone=False, psi_dtype=psi_dtype, tune=True,
               direct_per_cu=direct_per_cu)
        out["tuned_wall_s"] = t["wall_s"]
        out["tuned_tune_s"] = t["tune_s"]
        out["speedup_tuned_vs_default"] = secs / t["wall_s"]
    if compare_alone:
        _sync()
        t0 = time.perf_counter()
        alone = [solver.solve(p, **sh) for p, sh in zip(probs, shapes)]
        _sync()
        secs_a = time.perf_counter() - t0
        out["alone_wall_s"] = secs_a
        out["alone_solves_per_s"] = n_instances / secs_a
        out["speedup_vs_alone"] = secs_a / secs
        out["max_rel_diff_vs_alone"] = same_results(
            [dict(name=p.name, qoi_int=r["qoi_int"]) for p, r in zip(probs, res)],
            [dict(name=p.name, qoi_int=r["qoi_int"]) for p, r in zip(probs, alone)])
    if verbose:
        print(f"[uq] {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def sweep(n_requests: int = 24, rates=(0.5, 0.9), seed: int = 0, budget_gb: float = 200.0,
          dtypes=("f32", "bf16"), max_instances: int = 64, steps_per_run: int = 32,
          policies=("deadline", "srpt"), capacity_batched: bool = True, verbose: bool = False,
          capacity: float | None = None):
    """Capacity of both paths (all requests at once), then the one-at-a-time
    path and the continuous-batching loop (each policy) on the same Poisson
    arrivals at fractions of the one-at-a-time capacity. `capacity` (solves
    per second) fixes the rate scale instead of the measured one, so that
    sweeps split over several runs share it; the back-to-back service times
    (for the slowdowns) are measured either way."""
    base = I.serving_requests(n_requests, rate=1.0, seed=seed, dtypes=dtypes)
    # capacity: back-to-back service times of the plain path (arrivals all at 0)
    cap_reqs = [(0.0, p) for _, p in base]
    cap_rec, cap_tot = serve_fifo(cap_reqs, verbose=verbose)
    alone = {r["name"]: r["service"] for r in cap_rec}
    measured = len(cap_rec) / sum(alone.values())
    capacity = capacity or measured
    out = dict(requests=n_requests, capacity_solves_per_s=capacity, measured_capacity_solves_per_s=measured,
               mean_service_s=float(np.mean(list(alone.values()))), policies=list(policies),
               steps_per_run=steps_per_run, rates=[])
    if capacity_batched:
        rec_c, tot_c = serve(cap_reqs, int(budget_gb * 1e9), max_instances=max_instances,
                             steps_per_run=steps_per_run, policy=policies[0], verbose=verbose)
        out["capacity_batched_solves_per_s"] = len(rec_c) / tot_c["wall_s"]
        out["capacity_fifo_solves_per_s"] = len(cap_rec) / cap_tot["wall_s"]
    for f in rates:
        lam = f * capacity
        # same requests, arrival times rescaled to rate lam
        arr = [(t / lam, p) for t, p in base]
        rec_f, tot_f = serve_fifo(arr, verbose=verbose)
        entry = dict(load=f, rate_per_s=lam, fifo=summarize(rec_f, tot_f, alone))
        for pol in policies:
            rec_b, tot_b = serve(arr, int(budget_gb * 1e9), max_instances=max_instances,
                                 steps_per_run=steps_per_run, policy=pol, verbose=verbose)
            entry[f"batched_{pol}"] = summarize(rec_b, tot_b, alone)
            entry[f"max_rel_diff_{pol}_vs_fifo"] = same_results(rec_b, rec_f)
        out["rates"].append(entry)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--rates", default="0.25,0.5,0.75,0.9,1.1")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--uq", type=int, default=0, help="run the UQ batch with this many instances")
    ap.add_argument("--policies", default="deadline,srpt")
    ap.add_argument("--capacity", type=float, default=0.0, help="rate scale in solves/s (0: measure it)")
    ap.add_argument("--no-capacity-batched", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args(argv)
    res = {}
    if args.uq:
        res["uq"] = uq(args.uq, verbose=args.verbose)
    if args.requests:
        res["serving"] = sweep(args.requests, tuple(float(x) for x in args.rates.split(",")), args.seed,
                               args.budget_gb, policies=tuple(args.policies.split(",")),
                               capacity_batched=not args.no_capacity_batched, verbose=args.verbose,
                               capacity=args.capacity or None)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
