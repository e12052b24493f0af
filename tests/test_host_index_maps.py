"""Host-side checks of the hopping kernels' index maps (tests/host/index_maps.cpp): division by an
invariant divisor equals integer division for every divisor and position the z-range processing order
produces, and the y-z block order is a bijection of the sites that keeps each block inside its (y, z)
range.  The C++ file includes the library's own header, so the functions checked are the ones the
kernels run (here compiled for the host)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_index_maps_on_the_host(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = tmp_path / "index_maps"
    build = subprocess.run([HIPCC, "-O2", "-std=c++17", "--cuda-host-only", "-x", "hip",
                            "-I", os.path.join(ROOT, "include"),
                            "-I", os.path.join(ROOT, "paper_1405_0700_amd", "csrc"),
                            os.path.join(ROOT, "tests", "host", "index_maps.cpp"), "-o", str(exe)],
                           capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-2000:]
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert run.returncode == 0 and run.stdout.strip() == "ok", run.stdout
