"""Grouping of linear combinations over the same sources into multi-output
jobs (host logic of the executor, built with hipcc for the host, run on the
CPU): every output kept once with its weights, constant and destination;
different source lists never merge; the launch's cost counts."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_lincomb_grouping_on_host(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("no hipcc")
    exe = tmp_path / "lin_group_host"
    src = os.path.join(HERE, "native", "lin_group_host.cpp")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-x", "hip", "-o", str(exe), src],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok (4 jobs)"), r.stdout
