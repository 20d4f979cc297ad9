"""Per-solve driver: one plan, device buffers from PyTorch, the HIP library does the work.

    from paper_2505_17284_amd import inputs, solver
    r = solver.solve(inputs.config(2))      # QoIs of the 700^2 lattice, 256 ordinates

PyTorch only allocates device memory and supplies the stream; every stage of
the transport step runs in libsnrt's kernels (include/snrt.h).
"""

from __future__ import annotations

import ctypes

import numpy as np

from ._lib import (FLUENCE_PIECE, MAX_FLUENCE_BLOCKS, MAX_RECTS, MAX_TALLIES, SN_ERR_NONFINITE,
                   MarshalledProblem, SnError, SnPlanInfo, SnQoi, check, lib)


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the S_N transport library needs a ROCm GPU (torch.cuda is not available)")
    return torch


def plan_info(problem, group_size: int = 0, rows_per_wave: int = 0, waves_per_group: int = 0,
              group_size_average: int = 0, fluence: bool = False, probes=None) -> dict:
    """Derived constants and buffer sizes of a plan (host only, no GPU).
    group_size applies to both stages unless group_size_average is given."""
    m = MarshalledProblem(problem, fluence, probes)
    h = ctypes.c_void_p()
    check(lib().sn_plan_create_shaped(ctypes.byref(m.struct), group_size, group_size_average or group_size,
                                      rows_per_wave, waves_per_group, ctypes.byref(h)), "sn_plan_create")
    try:
        info = SnPlanInfo()
        check(lib().sn_plan_get_info(h, ctypes.byref(info)), "sn_plan_get_info")
        return {f: getattr(info, f) for f, _ in SnPlanInfo._fields_}
    finally:
        lib().sn_plan_destroy(h)


def qoi_dicts(problem, q: SnQoi):
    """(instantaneous, integrated) QoIs keyed like the oracle's names."""
    T, R = problem.n_tallies, problem.n_rects
    inst = {"mass": q.mass, "source": q.source}
    integ = {"mass": q.int_mass, "source": q.int_source}
    for t in range(T):
        inst[f"abs:{problem.tally_names[t]}"] = q.absorption[t]
        integ[f"abs:{problem.tally_names[t]}"] = q.int_absorption[t]
    for r in range(R):
        inst[f"out:{problem.rect_names[r]}"] = q.outflow[r]
        inst[f"in:{problem.rect_names[r]}"] = q.inflow[r]
        integ[f"out:{problem.rect_names[r]}"] = q.int_outflow[r]
        integ[f"in:{problem.rect_names[r]}"] = q.int_inflow[r]
    return inst, integ


class Plan:
    """A bound, initialised solve on one GPU."""

    def __init__(self, problem, group_size: int = 0, rows_per_wave: int = 0, waves_per_group: int = 0,
                 device: str = "cuda:0", psi0=None, graph_steps: int = 0, group_size_average: int = 0,
                 fluence: bool = False, probes=None, static_scratch: bool = False):
        """fluence: keep the time integral of phi per cell (``fluence()``);
        probes: space-time probes, a dict with n_probes, n_windows and cells
        (PROBE_CELL records; ``hohlraum.probe_cells`` builds the paper's);
        static_scratch: take the scratch from the library's own device area
        (sn_plan_bind_static) instead of a PyTorch buffer."""
        torch = _torch()
        assert problem.n_tallies <= MAX_TALLIES and problem.n_rects <= MAX_RECTS
        self.problem = problem
        self.device = torch.device(device)
        self._probes = probes
        self._m = MarshalledProblem(problem, fluence, probes)
        self.h = ctypes.c_void_p()
        check(lib().sn_plan_create_shaped(ctypes.byref(self._m.struct), group_size,
                                          group_size_average or group_size, rows_per_wave,
                                          waves_per_group, ctypes.byref(self.h)), "sn_plan_create")
        info = SnPlanInfo()
        check(lib().sn_plan_get_info(self.h, ctypes.byref(info)), "sn_plan_get_info")
        self.info = {f: getattr(info, f) for f, _ in SnPlanInfo._fields_}
        with torch.cuda.device(self.device):
            self.psi_a = torch.empty(int(info.psi_bytes), dtype=torch.uint8, device=self.device)
            self.psi_b = torch.empty(int(info.psi_bytes), dtype=torch.uint8, device=self.device)
            if static_scratch:
                self.scratch = None
                check(lib().sn_plan_bind_static(self.h, self.psi_a.data_ptr(), self.psi_b.data_ptr()),
                      "sn_plan_bind_static")
            else:
                self.scratch = torch.empty(int(info.scratch_bytes), dtype=torch.uint8, device=self.device)
                check(lib().sn_plan_bind(self.h, self.psi_a.data_ptr(), self.psi_b.data_ptr(),
                                         self.scratch.data_ptr()), "sn_plan_bind")
        if graph_steps:
            check(lib().sn_plan_use_graph(self.h, int(graph_steps)), "sn_plan_use_graph")
        self.init(psi0)

    @property
    def stream(self) -> int:
        torch = _torch()
        return torch.cuda.current_stream(self.device).cuda_stream

    @property
    def n_steps(self) -> int:
        return int(self.info["n_steps"])

    @property
    def dt(self) -> float:
        return float(self.info["dt"])

    def init(self, psi0=None):
        buf = None
        if psi0 is not None:
            buf = np.ascontiguousarray(np.asarray(psi0, dtype=np.float32).reshape(
                self.problem.M, self.problem.ny, self.problem.nx))
        ptr = buf.ctypes.data if buf is not None else None
        check(lib().sn_plan_init(self.h, ptr, self.stream), "sn_plan_init")

    def run(self, n_steps: int | None = None, unbounded: bool = False):
        n = self.n_steps if n_steps is None else int(n_steps)
        fn = lib().sn_plan_run_unbounded if unbounded else lib().sn_plan_run
        check(fn(self.h, n, self.stream), "sn_plan_run")

    def qoi(self, allow_nonfinite: bool = False):
        q = SnQoi()
        st = lib().sn_plan_qoi(self.h, ctypes.byref(q), self.stream)
        if not (allow_nonfinite and st == SN_ERR_NONFINITE):
            check(st, "sn_plan_qoi")
        inst, integ = qoi_dicts(self.problem, q)
        return dict(step=int(q.step), t=float(q.t), qoi=inst, qoi_int=integ,
                    balance_residual=float(q.balance_residual), nonfinite=bool(q.nonfinite))

    def psi(self) -> np.ndarray:
        p = self.problem
        out = np.empty((p.M, p.ny, p.nx), dtype=np.float32)
        check(lib().sn_plan_read_psi(self.h, out.ctypes.data, self.stream), "sn_plan_read_psi")
        return out

    def phi(self) -> np.ndarray:
        p = self.problem
        out = np.empty((p.ny, p.nx), dtype=np.float32)
        check(lib().sn_plan_read_phi(self.h, out.ctypes.data, self.stream), "sn_plan_read_phi")
        return out

    def probes(self) -> np.ndarray:
        """Window averages of the probes so far: [n_windows][n_probes][phi, J_x, J_y]."""
        if self._probes is None:
            raise SnError(7, "sn_plan_read_probes", "plan has no probes")
        out = np.empty((int(self._probes["n_windows"]), int(self._probes["n_probes"]), 3), dtype=np.float64)
        check(lib().sn_plan_read_probes(self.h, out.ctypes.data, self.stream), "sn_plan_read_probes")
        return out

    def fluence(self) -> np.ndarray:
        """Time integral of phi per cell since init ([ny][nx] float64); the
        plan must have been made with ``fluence=True``."""
        p = self.problem
        out = np.empty((p.ny, p.nx), dtype=np.float64)
        check(lib().sn_plan_read_fluence(self.h, out.ctypes.data, self.stream), "sn_plan_read_fluence")
        return out

    def fluence_functionals(self, pieces: np.ndarray, set_start: np.ndarray, n_blocks: int) -> dict:
        """Block and line functionals of sigma_a * fluence, on the device
        (sn_plan_fluence_functionals): A_G, V_G, A_L, V_L and the block means A."""
        torch = _torch()
        pieces = np.ascontiguousarray(pieces, dtype=FLUENCE_PIECE)
        set_start = np.ascontiguousarray(set_start, dtype=np.int32)
        if not 1 <= n_blocks <= MAX_FLUENCE_BLOCKS or set_start.shape != (n_blocks + 2,):
            raise ValueError("set_start must hold n_blocks + 2 entries, 1 <= n_blocks <= %d" % MAX_FLUENCE_BLOCKS)
        raw = torch.from_numpy(pieces.view(np.uint8).reshape(-1)).to(self.device) if len(pieces) else None
        ss = torch.from_numpy(set_start).to(self.device)
        out = torch.empty(4 + n_blocks, dtype=torch.float64, device=self.device)
        check(lib().sn_plan_fluence_functionals(self.h, raw.data_ptr() if raw is not None else None,
                                                int(len(pieces)), ss.data_ptr(), int(n_blocks),
                                                out.data_ptr(), self.stream), "sn_plan_fluence_functionals")
        o = out.cpu().numpy()
        return dict(A_G=float(o[0]), V_G=float(o[1]), A_L=float(o[2]), V_L=float(o[3]), A=o[4:].copy())

    def set_timing(self, on: bool):
        check(lib().sn_plan_set_timing(self.h, 1 if on else 0), "sn_plan_set_timing")

    def kernel_ms(self):
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int64 * 4)()
        check(lib().sn_plan_kernel_ms(self.h, ctypes.byref(ms), ctypes.byref(cnt)), "sn_plan_kernel_ms")
        return list(ms), list(cnt)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().sn_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(problem, steps: int | None = None, psi0=None, return_psi: bool = False, **plan_kw):
    """Run a problem to t_end (or ``steps`` steps) on the GPU and return its QoIs."""
    plan = Plan(problem, psi0=psi0, **plan_kw)
    try:
        plan.run(steps)
        r = plan.qoi()
        r["nt"], r["dt"] = plan.n_steps, plan.dt
        if return_psi:
            r["psi"] = plan.psi()
            r["phi"] = plan.phi()
        return r
    finally:
        plan.close()


_TUNED: dict = {}

# (update stage, averaging stage) ordinates per group tried by autotune; 0
# is the library's default for the shape.
TUNE_CANDIDATES = ((0, 0), (8, 8), (16, 16), (32, 16), (32, 32), (64, 32), (64, 64))


def autotune(problem, candidates=TUNE_CANDIDATES, steps: int = 4, reps: int = 2, device: str = "cuda:0") -> dict:
    """The fastest ordinate-group sizes for the problem's shape class (grid,
    ordinates, order, stepper, storage), measured on the device: for every
    distinct effective candidate, the best of `reps` wall-clock timings of
    `steps` whole steps (stages, finalizes, launches) after one warm-up step.
    Cached per class for the life of the process; returns group_size,
    group_size_average and the measured ms per step."""
    import time

    torch = _torch()
    key = (problem.nx, problem.ny, problem.M, problem.order, problem.stepper, problem.psi_dtype)
    if key in _TUNED:
        return _TUNED[key]
    best = None
    seen = set()
    for gs, gsa in candidates:
        info = plan_info(problem, group_size=gs, group_size_average=gsa or gs)
        eff = (info["group_size"], info["group_size_average"])
        if eff in seen:
            continue
        seen.add(eff)
        plan = Plan(problem, group_size=eff[0], group_size_average=eff[1], device=device)
        try:
            plan.run(1, unbounded=True)
            t = float("inf")
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan.run(steps, unbounded=True)
                torch.cuda.synchronize()
                t = min(t, (time.perf_counter() - t0) * 1e3 / steps)
        finally:
            plan.close()
        if best is None or t < best[0]:
            best = (t, eff)
    _TUNED[key] = dict(group_size=best[1][0], group_size_average=best[1][1], ms_per_step=best[0])
    return _TUNED[key]


__all__ = ["Plan", "solve", "plan_info", "qoi_dicts", "SnError", "autotune"]
