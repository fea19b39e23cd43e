"""The NTT pass logic (radix-16 register passes, LDS exchanges, global
layouts) under every radix split the batched kernel is compiled with, run on
the host thread by thread with the host compiler: the forward transform equals
a textbook negacyclic NTT at every index (evaluation at odd powers of psi),
every index is written once, the inverse returns the input, exchanges that
skip the workgroup barrier stay inside one wave, and the padded LDS placement is
one to one, in bounds and (at N = 16384) spreads each register access of the
strided passes over the banks."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_ntt_split_variants_on_host(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "ntt_split_host"
    src = os.path.join(HERE, "native", "ntt_split_host.cpp")
    subprocess.run([cxx, "-O2", "-std=c++17", "-Wno-unknown-pragmas", "-o", str(exe), src], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    lines = r.stdout.strip().splitlines()
    assert r.returncode == 0, r.stdout
    assert len(lines) == 26 and all(ln.endswith(": ok") for ln in lines)
