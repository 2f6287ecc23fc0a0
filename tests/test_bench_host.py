"""Host-side logic of bench.py (no GPU): the one-GPU guard, the guard that
drops the committed HBM traffic figure once the face kernel's sources have
changed, and the flop table lookup for every configuration bench.py runs."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_is_dropped_when_the_kernel_source_changes(monkeypatch, tmp_path):
    f = tmp_path / "traffic.txt"
    f.write_text("# comment\nkernel_source_sha = 0123456789abcdef\n"
                 "bytes_per_launch[turb128/fp64/q26] = 1234\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123456789abcdef")
    assert bench.read_traffic("turb128", "fp64", "q26") == 1234.0
    assert bench.read_traffic("turb128", "fp32", "q26") is None  # no entry for that form
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "fedcba9876543210")
    assert bench.read_traffic("turb128", "fp64", "q26") is None


def test_kernel_source_hash_covers_the_face_kernel_sources(monkeypatch, tmp_path):
    csrc = tmp_path / "paper_2609_10816_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.FACE_KERNEL_SOURCES:
        (csrc / name).write_text("x")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    (csrc / bench.FACE_KERNEL_SOURCES[1]).write_text("y")
    assert bench.kernel_source_hash() != h0


@pytest.mark.parametrize("name", sorted(bench.CONFIGS))
@pytest.mark.parametrize("emf", ["q26", "b25a", "fs18"])
def test_flop_table_has_every_bench_configuration(name, emf):
    cfg = bench.CONFIGS[name]
    tab = json.load(open(bench.FLOPS_FILE))["entries"]
    key = f"{cfg['recon']}/{emf}/eta{'>0' if cfg['eta'] > 0 else '=0'}"
    assert key in tab
    assert tab[key]["face_flops"] > 0 and tab[key]["cell_update_flops"] > tab[key]["face_flops"]


def test_cpu_model_is_read():
    name, n = bench.cpu_model()
    assert isinstance(name, str) and name and n >= 1


def test_default_workload_is_the_512_box():
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--config", default="turb512"' in src
    assert bench.CONFIGS["turb512"]["n"] == 512 and bench.CONFIGS["turb512"]["eta"] == 1e-3
