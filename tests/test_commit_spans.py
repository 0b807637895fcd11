"""Host check of the one-pass commit's index spans (`csrc/commit_span.h`, used by
the commit kernel): each stored voxel is written by exactly one workgroup, which
also loads it, and every macrocell window lies inside the loaded range of the
workgroup that reduces it.  Built with hipcc for the host and run on the CPU."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not installed")
def test_commit_spans(tmp_path):
    exe = tmp_path / "commit_span_check"
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
           "-I", os.path.join(ROOT, "paper_2407_00179_amd", "csrc"),
           os.path.join(ROOT, "tests", "native", "commit_span_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout
