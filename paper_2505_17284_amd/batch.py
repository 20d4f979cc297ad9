"""Batched solves: many independent S_N problems advanced together on one GPU.

    from paper_2505_17284_amd import inputs as I
    from paper_2505_17284_amd.batch import Batch

    b = Batch(max_instances=256, steps_per_run=16)
    slots = [b.admit(I.uq_instance(seed)) for seed in range(8)]
    while b.unfinished():
        b.run()
    results = [b.result(s) for s in slots]

Every admitted problem keeps its state in its own device buffers (allocated
through PyTorch when it is admitted). Each stage of all unfinished problems is
one persistent launch of the library's batched stage kernel, followed by one
batched finalize; the launches of a run are replayed from a captured hipGraph
while the admitted set and its active pattern repeat (include/snrt.h,
sn_batch_*). Admission is bounded by slots and by an HBM budget.
"""

from __future__ import annotations

import ctypes

from . import solver
from ._lib import SN_BF16, SN_ERR_BUSY, SN_F32, SnBatchInfo, SnBatchOpts, SnError, check, lib


PAUSED = -1  # step quota of a slot that takes no steps (SN_STEPS_PAUSED)


class Busy(RuntimeError):
    """No free slot or not enough budget for the problem right now."""


def footprint(problem, rows_per_wave: int = 0, waves_per_group: int = 0, group_size: int = 0,
              fluence: bool = False, probes=None, group_size_average: int = 0) -> int:
    """HBM bytes a problem occupies while admitted (two psi buffers + scratch); host only."""
    info = solver.plan_info(problem, group_size, rows_per_wave, waves_per_group, group_size_average,
                            fluence=fluence, probes=probes)
    return 2 * int(info["psi_bytes"]) + int(info["scratch_bytes"])


class Batch:
    def __init__(self, order: int = 2, stepper: int = 1, psi_dtype: str = "f32", max_instances: int = 256,
                 steps_per_run: int = 16, rows_per_wave: int = 2, waves_per_group: int = 4,
                 hbm_budget_bytes: int = 0, use_graph: bool = True, workgroups_per_cu: int = 0,
                 cache_group_bytes: int = 0, direct_min_workgroups: int = 0, device: str = "cuda:0"):
        torch = solver._torch()
        self.device = torch.device(device)
        self.opts = SnBatchOpts(max_instances=max_instances, max_steps_per_run=steps_per_run, order=order,
                                stepper=stepper, psi_dtype=SN_BF16 if psi_dtype == "bf16" else SN_F32,
                                rows_per_wave=rows_per_wave, waves_per_group=waves_per_group,
                                hbm_budget_bytes=hbm_budget_bytes, use_graph=1 if use_graph else 0,
                                workgroups_per_cu=workgroups_per_cu, cache_group_bytes=cache_group_bytes,
                                direct_min_workgroups=direct_min_workgroups)
        self.psi_dtype = psi_dtype
        self.steps_per_run = steps_per_run
        nbytes = ctypes.c_uint64()
        check(lib().sn_batch_workspace_bytes(ctypes.byref(self.opts), ctypes.byref(nbytes)), "sn_batch_workspace_bytes")
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            self.h = ctypes.c_void_p()
            check(lib().sn_batch_create(ctypes.byref(self.opts), self.workspace.data_ptr(), ctypes.byref(self.h)),
                  "sn_batch_create")
        self.plans: dict[int, solver.Plan] = {}
        self.bytes_admitted = 0

    @property
    def stream(self) -> int:
        torch = solver._torch()
        return torch.cuda.current_stream(self.device).cuda_stream

    def footprint(self, problem, group_size: int = 0, fluence: bool = False, probes=None,
                  group_size_average: int = 0) -> int:
        return footprint(problem, self.opts.rows_per_wave, self.opts.waves_per_group, group_size, fluence, probes,
                         group_size_average)

    def fits(self, problem, group_size: int = 0, fluence: bool = False, probes=None,
             group_size_average: int = 0) -> bool:
        if len(self.plans) >= self.opts.max_instances:
            return False
        if not self.opts.hbm_budget_bytes:
            return True
        return (self.bytes_admitted + self.footprint(problem, group_size, fluence, probes, group_size_average)
                <= self.opts.hbm_budget_bytes)

    def admit(self, problem, psi0=None, group_size: int = 0, fluence: bool = False, probes=None,
              group_size_average: int = 0) -> int:
        """Allocate, initialise and admit one problem; returns its slot. Raises Busy.
        With ``fluence`` / ``probes`` the slot's plan also accumulates the time
        integral of phi / the probes' window averages (``plan(slot)``).
        group_size / group_size_average: ordinates per workgroup of the update
        and averaging stages (0: the defaults; group_size alone sets both)."""
        if problem.psi_dtype != self.psi_dtype:
            raise ValueError(f"problem stores psi as {problem.psi_dtype}, the batch as {self.psi_dtype}")
        if not self.fits(problem, group_size, fluence, probes, group_size_average):
            raise Busy(f"{problem.name}: no slot or budget free")
        plan = solver.Plan(problem, group_size=group_size, rows_per_wave=self.opts.rows_per_wave,
                           waves_per_group=self.opts.waves_per_group, device=str(self.device), psi0=psi0,
                           fluence=fluence, probes=probes, group_size_average=group_size_average)
        slot = ctypes.c_int32(-1)
        st = lib().sn_batch_admit(self.h, plan.h, ctypes.byref(slot))
        if st == SN_ERR_BUSY:
            plan.close()
            raise Busy(lib().sn_last_error().decode(errors="replace"))
        if st != 0:
            plan.close()
            check(st, "sn_batch_admit")
        fp = ctypes.c_uint64()
        check(lib().sn_plan_footprint(plan.h, ctypes.byref(fp)), "sn_plan_footprint")
        self.bytes_admitted += int(fp.value)
        self.plans[slot.value] = plan
        return slot.value

    def run(self, n_steps: int | None = None):
        """Advance every unfinished admitted problem by up to n_steps (asynchronous)."""
        n = self.steps_per_run if n_steps is None else int(n_steps)
        check(lib().sn_batch_run(self.h, n, self.stream), "sn_batch_run")

    def synchronize(self):
        """Wait for every run issued so far."""
        solver._torch().cuda.synchronize(self.device)

    def set_steps(self, slot: int, steps: int):
        """Most steps the slot takes per run (0 = no quota, PAUSED = none until set again)."""
        check(lib().sn_batch_set_steps(self.h, slot, int(steps)), "sn_batch_set_steps")

    def status(self, slot: int):
        done = ctypes.c_int32()
        step = ctypes.c_int64()
        check(lib().sn_batch_status(self.h, slot, ctypes.byref(done), ctypes.byref(step)), "sn_batch_status")
        return bool(done.value), int(step.value)

    def done_slots(self):
        return [s for s in self.plans if self.status(s)[0]]

    def unfinished(self) -> int:
        info = SnBatchInfo()
        check(lib().sn_batch_get_info(self.h, ctypes.byref(info)), "sn_batch_get_info")
        return int(info.n_unfinished)

    def info(self) -> dict:
        info = SnBatchInfo()
        check(lib().sn_batch_get_info(self.h, ctypes.byref(info)), "sn_batch_get_info")
        return {f: getattr(info, f) for f, _ in SnBatchInfo._fields_}

    def plan(self, slot: int):
        """The plan admitted in ``slot`` (read-only use: the batch advances it)."""
        return self.plans[slot]

    def result(self, slot: int, psi: bool = False, allow_nonfinite: bool = False) -> dict:
        """QoIs of a slot's current state (synchronising), like solver.solve."""
        plan = self.plans[slot]
        r = plan.qoi(allow_nonfinite=allow_nonfinite)
        r["nt"], r["dt"] = plan.n_steps, plan.dt
        if psi:
            r["psi"] = plan.psi()
            r["phi"] = plan.phi()
        return r

    def retire(self, slot: int, keep: bool = False):
        """Free a slot. The plan (and its device memory) is released unless keep=True."""
        check(lib().sn_batch_retire(self.h, slot), "sn_batch_retire")
        plan = self.plans.pop(slot)
        fp = ctypes.c_uint64()
        check(lib().sn_plan_footprint(plan.h, ctypes.byref(fp)), "sn_plan_footprint")
        self.bytes_admitted -= int(fp.value)
        if keep:
            return plan
        plan.close()
        return None

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            for s in list(self.plans):
                self.retire(s)
            lib().sn_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_all(problems, max_instances: int | None = None, steps_per_run: int = 16, **kw):
    """Run every problem to its end time in one batch; returns their results in order."""
    if not problems:
        return []
    p0 = problems[0]
    b = Batch(order=p0.order, stepper=p0.stepper, psi_dtype=p0.psi_dtype,
              max_instances=max_instances or len(problems), steps_per_run=steps_per_run, **kw)
    try:
        slots = [b.admit(p) for p in problems]
        while b.unfinished():
            b.run()
        return [b.result(s) for s in slots]
    finally:
        b.close()


__all__ = ["Batch", "Busy", "PAUSED", "footprint", "solve_all", "SnError"]
