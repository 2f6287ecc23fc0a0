"""The C ABI from plain C: tests/abi_c_example.c includes only ctmhd.h and
the HIP runtime API and links libctmhd.so.  On the CPU it must compile and
link; on the GPU it runs one ctmhd_step call of 5 steps on a 16 x 12 x 8 box
(a uniform moving state stays bitwise fixed; a density wave conserves mass
and energy to 1e-13)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2609_10816_amd")


def _build(tmp_path):
    exe = tmp_path / "abi_c_example"
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
           os.path.join(ROOT, "tests", "abi_c_example.c"), "-o", str(exe),
           "-L", PKG, "-lctmhd", "-L", "/opt/rocm/lib", "-lamdhip64", "-lm",
           f"-Wl,-rpath,{PKG}", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_c_caller_compiles_and_links(tmp_path):
    assert os.path.exists(os.path.join(PKG, "libctmhd.so")), "build the library first"
    _build(tmp_path)


@pytest.mark.gpu
def test_c_caller_runs(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
