"""Host logic of the HIP library that needs no GPU: the 64-bit reciprocal
division the simulation kernels use to map run indices to (setting, trial)
and decision steps to histogram bins."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_udiv_magic_matches_plain_division(tmp_path):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "udiv_check")
    subprocess.run([HIPCC, "-O2", "-std=c++17", os.path.join(HERE, "helpers", "udiv_check.hip"),
                    "-o", exe], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    assert r.stdout.strip().endswith("bad 0")
