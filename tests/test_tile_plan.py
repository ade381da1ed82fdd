"""Host-side checks of the substep's tile plan (every tile of the grid
launched exactly once, interior boxes that reach no wall, disjoint
partial-result slots) and of its z-metric tables, by compiling and running
tests/hostcheck/tile_plan_check.cpp against the library's own header (host
code only: no device call).  CPU only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_tile_plan_partition_and_metric_tables(tmp_path):
    exe = tmp_path / "tile_plan_check"
    subprocess.check_call([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I",
                           os.path.join(ROOT, "paper_2502_04189_amd", "csrc"),
                           os.path.join(HERE, "hostcheck", "tile_plan_check.cpp"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
