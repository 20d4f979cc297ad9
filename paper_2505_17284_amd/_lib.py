"""ctypes binding of libsnrt.so (include/snrt.h): argument marshalling only.

Every step of the transport path runs in the library's HIP kernels. Loading
fails loudly when the library has not been built; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnrt.so")

SN_OK = 0
SN_ERR_INVALID = 1
SN_ERR_OOM = 2
SN_ERR_DEVICE = 3
SN_ERR_UNSUPPORTED = 4
SN_ERR_NONFINITE = 5
SN_ERR_BUSY = 6
SN_ERR_STATE = 7
SN_F32 = 0
SN_BF16 = 1
STATIC_SCRATCH_BYTES = 64 << 20  # SN_STATIC_SCRATCH_BYTES
MAX_TALLIES = 8
MAX_RECTS = 4
MAX_FLUENCE_BLOCKS = 1024
# sn_fluence_piece: two interior cell indices and the piece's weight
FLUENCE_PIECE = np.dtype([("cell_a", np.int32), ("cell_b", np.int32), ("weight", np.float64)])
# sn_probe_cell: interior cell index, probe id, the cell's weight in the probe's average
PROBE_CELL = np.dtype([("cell", np.int32), ("probe", np.int32), ("weight", np.float64)])
MAX_PROBES = 8

# Every symbol the header declares; tests check the library exports them all.
EXPORTED = [
    "sn_plan_create", "sn_plan_create_tuned", "sn_plan_create_shaped", "sn_plan_get_info", "sn_plan_bind",
    "sn_plan_bind_static",
    "sn_plan_init", "sn_plan_run", "sn_plan_run_unbounded", "sn_plan_qoi",
    "sn_plan_read_psi", "sn_plan_read_phi", "sn_plan_read_fluence", "sn_plan_fluence_functionals",
    "sn_plan_read_probes",
    "sn_plan_use_graph", "sn_plan_set_timing",
    "sn_plan_kernel_ms", "sn_plan_destroy", "sn_status_str", "sn_last_error",
    "sn_batch_workspace_bytes", "sn_batch_create", "sn_plan_footprint", "sn_batch_admit", "sn_batch_run",
    "sn_batch_set_steps", "sn_batch_status", "sn_batch_retire", "sn_batch_get_info", "sn_batch_destroy",
]

_d = ctypes.c_double
_i32 = ctypes.c_int32
_vp = ctypes.c_void_p


class SnProblem(ctypes.Structure):
    _fields_ = [
        ("nx", _i32), ("ny", _i32), ("h", _d), ("M", _i32),
        ("xi", _vp), ("eta", _vp), ("w", _vp), ("mirror_x", _vp), ("mirror_y", _vp),
        ("region", _vp), ("n_regions", _i32), ("sigma_a", _vp), ("sigma_s", _vp), ("q", _vp),
        ("tally", _vp), ("n_tallies", _i32), ("bc", _i32 * 4), ("inflow", _d * 4),
        ("order", _i32), ("stepper", _i32), ("cfl", _d), ("t_end", _d),
        ("n_rects", _i32), ("rects", _vp), ("psi_dtype", _i32), ("fluence", _i32),
        ("n_probes", _i32), ("n_windows", _i32), ("n_probe_cells", _i32), ("probe_cells", _vp),
    ]


class SnPlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_steps", _i32), ("dt", _d), ("nx", _i32), ("ny", _i32), ("M", _i32), ("pitch", _i32),
        ("n_groups", _i32), ("group_size", _i32), ("rows_per_wave", _i32), ("waves_per_group", _i32),
        ("n_workgroups", _i32),
        ("psi_bytes", ctypes.c_uint64), ("scratch_bytes", ctypes.c_uint64), ("psi_dtype", _i32),
        ("step", _i32), ("n_groups_average", _i32), ("group_size_average", _i32),
        ("n_workgroups_average", _i32),
    ]


class SnQoi(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("t", _d), ("n_tallies", _i32), ("n_rects", _i32),
        ("mass", _d), ("source", _d), ("absorption", _d * MAX_TALLIES),
        ("outflow", _d * MAX_RECTS), ("inflow", _d * MAX_RECTS),
        ("int_mass", _d), ("int_source", _d), ("int_absorption", _d * MAX_TALLIES),
        ("int_outflow", _d * MAX_RECTS), ("int_inflow", _d * MAX_RECTS),
        ("balance_residual", _d), ("nonfinite", _i32),
    ]


class SnBatchOpts(ctypes.Structure):
    _fields_ = [
        ("max_instances", _i32), ("max_steps_per_run", _i32), ("order", _i32), ("stepper", _i32),
        ("psi_dtype", _i32), ("rows_per_wave", _i32), ("waves_per_group", _i32),
        ("hbm_budget_bytes", ctypes.c_uint64), ("use_graph", _i32), ("workgroups_per_cu", _i32),
        ("cache_group_bytes", ctypes.c_uint64), ("direct_min_workgroups", _i32),
    ]


class SnBatchInfo(ctypes.Structure):
    _fields_ = [
        ("n_admitted", _i32), ("n_unfinished", _i32), ("bytes_admitted", ctypes.c_uint64),
        ("hbm_budget_bytes", ctypes.c_uint64), ("launches", ctypes.c_int64), ("graph_replays", ctypes.c_int64),
    ]


class SnError(RuntimeError):
    def __init__(self, status: int, where: str, text: str):
        super().__init__(f"{where}: status {status}: {text}")
        self.status = status


_lib = None


def lib():
    """The loaded library; raises if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (paper_2505_17284_amd/build.py)")
        # One HIP runtime per process: PyTorch, which supplies the device memory
        # and streams, ships its own libamdhip64 with the same soname. Loading it
        # first makes the library bind to that copy instead of a second runtime.
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        PP = ctypes.POINTER(_vp)
        L.sn_plan_create.argtypes = [ctypes.POINTER(SnProblem), PP]
        L.sn_plan_create_tuned.argtypes = [ctypes.POINTER(SnProblem), _i32, _i32, _i32, PP]
        L.sn_plan_create_shaped.argtypes = [ctypes.POINTER(SnProblem), _i32, _i32, _i32, _i32, PP]
        L.sn_plan_get_info.argtypes = [_vp, ctypes.POINTER(SnPlanInfo)]
        L.sn_plan_bind.argtypes = [_vp, _vp, _vp, _vp]
        L.sn_plan_bind_static.argtypes = [_vp, _vp, _vp]
        L.sn_plan_init.argtypes = [_vp, _vp, _vp]
        L.sn_plan_run.argtypes = [_vp, _i32, _vp]
        L.sn_plan_run_unbounded.argtypes = [_vp, _i32, _vp]
        L.sn_plan_qoi.argtypes = [_vp, ctypes.POINTER(SnQoi), _vp]
        L.sn_plan_read_psi.argtypes = [_vp, _vp, _vp]
        L.sn_plan_read_phi.argtypes = [_vp, _vp, _vp]
        L.sn_plan_read_fluence.argtypes = [_vp, _vp, _vp]
        L.sn_plan_read_probes.argtypes = [_vp, _vp, _vp]
        L.sn_plan_fluence_functionals.argtypes = [_vp, _vp, _i32, _vp, _i32, _vp, _vp]
        L.sn_plan_use_graph.argtypes = [_vp, _i32]
        L.sn_plan_set_timing.argtypes = [_vp, _i32]
        L.sn_plan_kernel_ms.argtypes = [_vp, ctypes.POINTER(_d * 4), ctypes.POINTER(ctypes.c_int64 * 4)]
        L.sn_plan_destroy.argtypes = [_vp]
        L.sn_plan_destroy.restype = None
        L.sn_batch_workspace_bytes.argtypes = [ctypes.POINTER(SnBatchOpts), ctypes.POINTER(ctypes.c_uint64)]
        L.sn_batch_create.argtypes = [ctypes.POINTER(SnBatchOpts), _vp, PP]
        L.sn_plan_footprint.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint64)]
        L.sn_batch_admit.argtypes = [_vp, _vp, ctypes.POINTER(_i32)]
        L.sn_batch_run.argtypes = [_vp, _i32, _vp]
        L.sn_batch_set_steps.argtypes = [_vp, _i32, _i32]
        L.sn_batch_status.argtypes = [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_int64)]
        L.sn_batch_retire.argtypes = [_vp, _i32]
        L.sn_batch_get_info.argtypes = [_vp, ctypes.POINTER(SnBatchInfo)]
        L.sn_batch_destroy.argtypes = [_vp]
        L.sn_batch_destroy.restype = None
        L.sn_status_str.argtypes = [_i32]
        L.sn_status_str.restype = ctypes.c_char_p
        L.sn_last_error.argtypes = []
        L.sn_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            fn = getattr(L, name)
            if fn.restype is ctypes.c_int:  # default restype: every status-returning call
                fn.restype = _i32
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != SN_OK:
        raise SnError(status, where, lib().sn_last_error().decode(errors="replace"))


class MarshalledProblem:
    """A problem statement laid out as the C struct, owning contiguous copies."""

    def __init__(self, p, fluence: bool = False, probes=None):
        """probes: None, or a dict with n_probes, n_windows and cells (an array
        of PROBE_CELL records)."""
        qd = p.quad
        self.keep = dict(
            xi=np.ascontiguousarray(qd.xi, np.float64), eta=np.ascontiguousarray(qd.eta, np.float64),
            w=np.ascontiguousarray(qd.w, np.float64),
            mirror_x=np.ascontiguousarray(qd.mirror_x, np.int32),
            mirror_y=np.ascontiguousarray(qd.mirror_y, np.int32),
            region=np.ascontiguousarray(p.region, np.uint8),
            sigma_a=np.ascontiguousarray(p.sigma_a, np.float64),
            sigma_s=np.ascontiguousarray(p.sigma_s, np.float64),
            q=np.ascontiguousarray(p.q, np.float64), tally=np.ascontiguousarray(p.tally, np.uint8),
            rects=np.ascontiguousarray(np.asarray(p.rects, np.int32).reshape(-1, 4)),
        )
        k = self.keep
        s = SnProblem()
        s.nx, s.ny, s.h, s.M = int(p.nx), int(p.ny), float(p.h), int(k["w"].shape[0])
        for name in ("xi", "eta", "w", "mirror_x", "mirror_y", "region", "sigma_a", "sigma_s",
                     "q", "tally", "rects"):
            setattr(s, name, k[name].ctypes.data)
        s.n_regions = int(k["sigma_a"].shape[0])
        s.n_tallies = int(len(p.tally_names))
        s.bc = (_i32 * 4)(*[int(b) for b in p.bc])
        s.inflow = (_d * 4)(*[float(g) for g in p.inflow])
        s.order, s.stepper = int(p.order), int(p.stepper)
        s.cfl, s.t_end = float(p.cfl), float(p.t_end)
        s.n_rects = int(k["rects"].shape[0])
        s.psi_dtype = SN_BF16 if p.psi_dtype == "bf16" else SN_F32
        s.fluence = 1 if fluence else 0
        if probes is not None:
            cells = np.ascontiguousarray(probes["cells"], dtype=PROBE_CELL)
            self.keep["probe_cells"] = cells
            s.n_probes, s.n_windows = int(probes["n_probes"]), int(probes["n_windows"])
            s.n_probe_cells = int(cells.shape[0])
            s.probe_cells = cells.ctypes.data if cells.shape[0] else None
        self.struct = s
