"""Build libsnrt.so (the HIP kernels and the C ABI) in-tree for gfx950."""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsnrt.so")
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in (
    "sn_stage_o1_f32.hip", "sn_stage_o2_f32.hip", "sn_stage_o1_bf16.hip", "sn_stage_o2_bf16.hip",
    "sn_stage_o3_f32.hip", "sn_stage_o3_bf16.hip",
    "sn_aux.hip", "snrt_plan.cpp", "snrt_batch.cpp", "snrt_static.hip")]
ARCH = os.environ.get("SNRT_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay off (see the design notes)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _filter(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source for gfx950 (in parallel) and link libsnrt.so next to this file."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + f".{os.getpid()}.o")
        cmd = [hipcc(), f"--offload-arch={ARCH}", *FLAGS, *inc, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, r.returncode, _filter(r.stdout + r.stderr), cmd

    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)), 16)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(compile_one, SOURCES))
    for src, obj, rc, out, cmd in results:
        if verbose:
            print(" ".join(cmd), flush=True)
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)} ({rc}):\n{out}")
        if verbose and out.strip():
            print(out, file=sys.stderr)
    tmp = LIB + f".tmp{os.getpid()}"
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *[o for _, o, _, _, _ in results], "-o", tmp]
    r = subprocess.run(link, capture_output=True, text=True)
    for _, o, _, _, _ in results:
        os.remove(o)
    if r.returncode != 0:
        raise RuntimeError(f"link failed ({r.returncode}):\n{_filter(r.stdout + r.stderr)}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
