"""Block -> (job, unit) mappings of the batched key-switch kernels (host
build of the same functions the kernels call): each unit of each job runs
exactly once, jobs stay on their XCD's range, and long units are handed out
ahead of short ones."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_xcd_job_unit_mappings_on_host(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("no hipcc")
    exe = tmp_path / "xcd_map_host"
    src = os.path.join(HERE, "native", "xcd_map_host.cpp")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-x", "hip",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", os.path.join(HERE, "..", "include"), "-o", str(exe), src],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().startswith("ok"), r.stdout
