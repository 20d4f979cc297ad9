"""FP64 CPU oracle for the explicit S_N transport step (test infrastructure).

TEST INFRASTRUCTURE ONLY: the parity tests, the smoke check and the
benchmark's CPU-baseline leg are the only users. The product path never
imports, links or runs anything here, and nothing here imports the product
package: problems are passed in as plain objects with numpy attributes (the
``Problem`` statements built by the seeded input generators).

The arithmetic lives in ``sn_oracle.c`` (plain C, FP64, loops in the order of
the paper's equations); this module only marshals arguments with ctypes.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sn_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsn_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, -O2, OpenMP over ordinates)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Prob(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("h", ctypes.c_double),
        ("M", ctypes.c_int),
        ("xi", ctypes.c_void_p), ("eta", ctypes.c_void_p), ("w", ctypes.c_void_p),
        ("mirror_x", ctypes.c_void_p), ("mirror_y", ctypes.c_void_p),
        ("region", ctypes.c_void_p), ("n_regions", ctypes.c_int),
        ("sigma_a", ctypes.c_void_p), ("sigma_s", ctypes.c_void_p), ("q", ctypes.c_void_p),
        ("tally", ctypes.c_void_p), ("n_tallies", ctypes.c_int),
        ("bc", ctypes.c_int * 4), ("inflow", ctypes.c_double * 4),
        ("order", ctypes.c_int), ("stepper", ctypes.c_int),
        ("cfl", ctypes.c_double), ("t_end", ctypes.c_double),
        ("n_rects", ctypes.c_int), ("rects", ctypes.c_void_p),
    ]


class _Probes(ctypes.Structure):
    _fields_ = [
        ("n_probes", ctypes.c_int), ("n_windows", ctypes.c_int), ("n_cells", ctypes.c_int),
        ("cell_i", ctypes.c_void_p), ("cell_j", ctypes.c_void_p), ("probe", ctypes.c_void_p),
        ("weight", ctypes.c_void_p),
    ]


class _MarshalledProbes:
    """probes: dict with n_probes, n_windows and per-cell arrays cell_i,
    cell_j, probe, weight (see oracle.hohlraum_qoi.probe_cells)."""

    def __init__(self, pr):
        self.arrs = dict(cell_i=np.ascontiguousarray(pr["cell_i"], np.int32),
                         cell_j=np.ascontiguousarray(pr["cell_j"], np.int32),
                         probe=np.ascontiguousarray(pr["probe"], np.int32),
                         weight=np.ascontiguousarray(pr["weight"], np.float64))
        s = _Probes()
        s.n_probes, s.n_windows = int(pr["n_probes"]), int(pr["n_windows"])
        s.n_cells = int(self.arrs["weight"].shape[0])
        for k, a in self.arrs.items():
            setattr(s, k, a.ctypes.data)
        self.s = s
        self.ref = ctypes.byref(s)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_Prob)
        d = ctypes.c_void_p
        lib.orc_threads.argtypes = [ctypes.c_int]
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_num_steps.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
        lib.orc_num_steps.restype = ctypes.c_int
        lib.orc_scalar_flux.argtypes = [P, d, d]
        lib.orc_face_x.argtypes = [P, d, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_face_x.restype = ctypes.c_double
        lib.orc_face_y.argtypes = [P, d, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_face_y.restype = ctypes.c_double
        lib.orc_rhs.argtypes = [P, d, d, d]
        lib.orc_qoi_len.argtypes = [P]
        lib.orc_qoi_len.restype = ctypes.c_int
        lib.orc_qoi.argtypes = [P, d, d, d]
        lib.orc_advance.argtypes = [P, ctypes.c_int, d, d, d, ctypes.POINTER(_Probes), ctypes.c_int, d]
        lib.orc_advance.restype = ctypes.c_int
        _lib = lib
    return _lib


class _Marshalled:
    """Keeps the contiguous copies alive while the C struct points at them."""

    def __init__(self, p):
        qd = p.quad
        self.arrs = dict(
            xi=np.ascontiguousarray(qd.xi, np.float64),
            eta=np.ascontiguousarray(qd.eta, np.float64),
            w=np.ascontiguousarray(qd.w, np.float64),
            mirror_x=np.ascontiguousarray(qd.mirror_x, np.int32),
            mirror_y=np.ascontiguousarray(qd.mirror_y, np.int32),
            region=np.ascontiguousarray(p.region, np.uint8),
            sigma_a=np.ascontiguousarray(p.sigma_a, np.float64),
            sigma_s=np.ascontiguousarray(p.sigma_s, np.float64),
            q=np.ascontiguousarray(p.q, np.float64),
            tally=np.ascontiguousarray(p.tally, np.uint8),
            rects=np.ascontiguousarray(np.asarray(p.rects).reshape(-1, 4), np.int32),
        )
        a = self.arrs
        s = _Prob()
        s.nx, s.ny, s.h, s.M = int(p.nx), int(p.ny), float(p.h), int(a["w"].shape[0])
        for k in ("xi", "eta", "w", "mirror_x", "mirror_y", "region", "sigma_a",
                  "sigma_s", "q", "tally", "rects"):
            setattr(s, k, a[k].ctypes.data)
        s.n_regions = int(a["sigma_a"].shape[0])
        s.n_tallies = int(len(p.tally_names))
        s.bc = (ctypes.c_int * 4)(*[int(b) for b in p.bc])
        s.inflow = (ctypes.c_double * 4)(*[float(g) for g in p.inflow])
        s.order, s.stepper = int(p.order), int(p.stepper)
        s.cfl, s.t_end = float(p.cfl), float(p.t_end)
        s.n_rects = int(a["rects"].shape[0])
        self.s = s
        self.ref = ctypes.byref(s)
        self.M, self.nx, self.ny = s.M, s.nx, s.ny


def threads(n: int = 0) -> int:
    """Set (n > 0) and return the number of OpenMP threads the oracle uses."""
    return int(_load().orc_threads(int(n)))


def num_steps(p):
    dt = ctypes.c_double(0.0)
    nt = _load().orc_num_steps(_Marshalled(p).ref, ctypes.byref(dt))
    return int(nt), float(dt.value)


def _state(m, psi):
    a = np.ascontiguousarray(np.asarray(psi, dtype=np.float64).reshape(m.M, m.ny, m.nx))
    return a


def scalar_flux(p, psi):
    m = _Marshalled(p)
    a = _state(m, psi)
    phi = np.zeros((m.ny, m.nx))
    _load().orc_scalar_flux(m.ref, a.ctypes.data, phi.ctypes.data)
    return phi


def rhs(p, psi):
    """F(psi) of the semi-discrete system."""
    m = _Marshalled(p)
    a = _state(m, psi)
    phi = scalar_flux(p, a)
    F = np.zeros_like(a)
    _load().orc_rhs(m.ref, a.ctypes.data, phi.ctypes.data, F.ctypes.data)
    return F


def face_x(p, psi, k, f, j):
    m = _Marshalled(p)
    a = _state(m, psi)
    return float(_load().orc_face_x(m.ref, a.ctypes.data, int(k), int(f), int(j)))


def face_y(p, psi, k, i, f):
    m = _Marshalled(p)
    a = _state(m, psi)
    return float(_load().orc_face_y(m.ref, a.ctypes.data, int(k), int(i), int(f)))


def qoi_names(p):
    names = ["mass", "source"]
    names += [f"abs:{t}" for t in p.tally_names]
    names += [f"out:{r}" for r in p.rect_names]
    names += [f"in:{r}" for r in p.rect_names]
    return names


def qoi(p, psi):
    """Instantaneous QoI vector of a state (see ``qoi_names``)."""
    m = _Marshalled(p)
    a = _state(m, psi)
    phi = scalar_flux(p, a)
    L = _load().orc_qoi_len(m.ref)
    qv = np.zeros(L)
    _load().orc_qoi(m.ref, a.ctypes.data, phi.ctypes.data, qv.ctypes.data)
    return qv


def advance(p, psi, n_steps, qint=None, fluence=None, probes=None, step0=0, probe_acc=None):
    """Advance a copy of ``psi`` by ``n_steps``; returns (psi, qint).

    With ``fluence`` (an [ny][nx] array, updated in place) the time integral
    of phi over the steps is added to it with the stepper's rule. With
    ``probes`` and ``probe_acc`` ([n_windows][n_probes][3], updated in place)
    the probes' window averages of phi, J_x, J_y are accumulated; ``step0`` is
    the index of the first step taken (it decides the windows).
    """
    m = _Marshalled(p)
    a = _state(m, psi).copy()
    L = _load().orc_qoi_len(m.ref)
    qi = np.zeros(L) if qint is None else np.array(qint, dtype=np.float64)
    fl = None
    if fluence is not None:
        if fluence.shape != (m.ny, m.nx) or fluence.dtype != np.float64 or not fluence.flags.c_contiguous:
            raise ValueError("fluence must be a C-contiguous float64 [ny][nx] array")
        fl = fluence.ctypes.data
    mp, pa = None, None
    if probes is not None:
        mp = _MarshalledProbes(probes)
        shape = (mp.s.n_windows, mp.s.n_probes, 3)
        if probe_acc is None or probe_acc.shape != shape or probe_acc.dtype != np.float64 \
                or not probe_acc.flags.c_contiguous:
            raise ValueError("probe_acc must be a C-contiguous float64 array of shape %s" % (shape,))
        pa = probe_acc.ctypes.data
    rc = _load().orc_advance(m.ref, int(n_steps), a.ctypes.data, qi.ctypes.data, fl,
                             mp.ref if mp is not None else None, int(step0), pa)
    if rc != 0:
        raise MemoryError("oracle could not allocate its work arrays")
    return a, qi


def solve(p, steps=None, psi0=None, fluence=False, probes=None):
    """Run the problem from psi0 (default 0) for ``steps`` (default N_t) steps.

    Returns a dict: psi, phi, nt, dt, steps, t, qoi (instantaneous at the end),
    qoi_int (time integrals), names, seconds, with ``fluence`` the time
    integral of phi per cell ("fluence", [ny][nx]), and with ``probes`` the
    probes' window averages ("probes", [n_windows][n_probes][phi, J_x, J_y]).
    """
    nt, dt = num_steps(p)
    steps = nt if steps is None else int(steps)
    if psi0 is None:
        psi0 = np.zeros((p.quad.M, p.ny, p.nx))
    fl = np.zeros((p.ny, p.nx)) if fluence else None
    pacc = None if probes is None else np.zeros((int(probes["n_windows"]), int(probes["n_probes"]), 3))
    t0 = time.perf_counter()
    psi, qint = advance(p, psi0, steps, fluence=fl, probes=probes, probe_acc=pacc)
    secs = time.perf_counter() - t0
    out = dict(psi=psi, phi=scalar_flux(p, psi), nt=nt, dt=dt, steps=steps,
               t=steps * dt, qoi=qoi(p, psi), qoi_int=qint, names=qoi_names(p),
               seconds=secs)
    if fluence:
        out["fluence"] = fl
    if probes is not None:
        out["probes"] = pacc
    return out
