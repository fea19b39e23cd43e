"""Two-prime conversions of key switching (host build of the device
functions the kernels call): a digit of two primes reduced mod another
modulus, and the centred lift over two special primes, against exact 128-bit
integer values; and the digit shapes (every ciphertext prime in exactly one
digit of at most K primes)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_two_prime_conversions_on_host(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("no hipcc")
    exe = tmp_path / "garner_host"
    src = os.path.join(HERE, "native", "garner_host.cpp")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-x", "hip",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", os.path.join(HERE, "..", "include"), "-o", str(exe), src],
                   check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().startswith("ok"), r.stdout
