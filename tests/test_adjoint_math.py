"""The reverse-mode per-point arithmetic of the HIP path (limiter, fast speed,
ideal-MHD flux, LLF, HLLD with alpha+-, u*, LD04 with Q26 corners) against
central finite differences of its own forward arithmetic, on the CPU: the
shared header is compiled as host code by hipcc and run here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
def test_adjoint_per_point_math_vs_finite_differences(tmp_path):
    exe = str(tmp_path / "adjoint_math_check")
    subprocess.check_call([HIPCC, "-O1", "-std=c++17", "-ffp-contract=off",
                           "-I", os.path.join(ROOT, "paper_2609_10816_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "adjoint_math_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "ALL OK" in r.stdout
