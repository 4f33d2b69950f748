"""Host-side checks of native helpers (compiled with g++, no GPU)."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_fastdiv_matches_hardware_division(tmp_path):
    exe = tmp_path / "fastdiv_check"
    src = os.path.join(ROOT, "tests", "native", "fastdiv_check.cpp")
    inc = os.path.join(ROOT, "paper_1103_6031_amd", "csrc")
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-I", inc, src, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout
    assert "mismatches 0" in r.stdout


def test_storage_index_maps_are_bijections(tmp_path):
    """lidx / ldecode (natural and colour-split layouts) round-trip on every cell of many shapes."""
    exe = tmp_path / "layout_check"
    src = os.path.join(ROOT, "tests", "native", "layout_check.cpp")
    inc = os.path.join(ROOT, "paper_1103_6031_amd", "csrc")
    r = subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", inc, src,
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert "mismatches 0" in r.stdout, r.stdout + r.stderr
    assert r.returncode == 0
