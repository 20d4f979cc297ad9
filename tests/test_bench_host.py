"""bench.py's host-side pieces, without a GPU: the algorithmic byte counts it
prices the kernels with, the refusal of more than one GPU, and the parsing of
the committed rocprofv3 summaries (values tied to the sources they measured)."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2505_17284_amd import inputs as I  # noqa: E402


def test_algorithmic_bytes_of_the_cavity_stages():
    """Per cell-ordinate 2 s (update stage) and 3 s (averaging stage) bytes,
    plus 9 bytes per cell (incoming and outgoing scalar flux, region id)."""
    p = I.config(3)
    cells, M = 1300 * 1300, 512
    assert bench.algorithmic_bytes(p, None, 1) == cells * M * 8 + 9 * cells == 6937450000
    assert bench.algorithmic_bytes(p, None, 2) == cells * M * 12 + 9 * cells == 10398570000
    b = p.replace(psi_dtype="bf16")
    assert bench.algorithmic_bytes(b, None, 2) == cells * M * 6 + 9 * cells


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("workload,dtype", [(bench.HEADLINE, "f32"), (bench.HEADLINE, "bf16"),
                                            ("lattice700_M256_heun2", "f32")])
def test_profile_summaries_parse(workload, dtype, tmp_path, monkeypatch):
    """The summary a workload names exists and carries its source hash; the
    traffic it records is read back only while the sources hash to it."""
    base = workload[: -len("_heun2")]
    path = os.path.join(bench.PROFILES, f"stage_heun2_{base}_{dtype}.md")
    assert os.path.exists(path)
    text = open(path).read()
    assert "source_sha256:" in text and "traffic_bytes_per_launch:" in text
    v = bench.measured_traffic(workload, dtype)
    if v is not None:  # the committed sources are the profiled ones
        assert v > bench.algorithmic_bytes(I.config(3) if "cavity" in workload else I.config(2),
                                           None, 2) * (0.5 if dtype == "bf16" else 1.0) * 0.9
    # a summary taken on other sources is not used
    fake = tmp_path / f"stage_heun2_{base}_{dtype}.md"
    fake.write_text(text.replace("source_sha256: `", "source_sha256: `0"))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.measured_traffic(workload, dtype) is None
