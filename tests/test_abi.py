"""The C-ABI library loads and exports every symbol include/lola.h declares;
parameter validation is host logic and runs without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lola.h")
LIB = os.path.join(ROOT, "paper_1812_10659_amd", "liblola.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lola_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1812_10659_amd import build_lib
        build_lib.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ["lola_ctx_create", "lola_keygen_secret", "lola_encode", "lola_encrypt", "lola_decrypt",
                 "lola_add", "lola_mul_plain", "lola_mul", "lola_relin", "lola_rotate"]:
        assert name in fns


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_galois_element_host_logic(lib):
    lib.lola_galois_element.restype = ctypes.c_uint32
    lib.lola_galois_element.argtypes = [ctypes.c_uint32, ctypes.c_int32]
    assert lib.lola_galois_element(16384, 1) == 3
    assert lib.lola_galois_element(16384, 0x7FFFFFFF) == 2 * 16384 - 1
    assert lib.lola_galois_element(16384, -1) == pow(3, 8191, 32768)
    assert lib.lola_galois_element(1000, 1) == 0


class _Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("t", ctypes.c_uint32), ("L", ctypes.c_uint32),
                ("q", ctypes.POINTER(ctypes.c_uint32)), ("P", ctypes.c_uint32), ("allow_insecure", ctypes.c_int),
                ("P2", ctypes.c_uint32)]


@pytest.mark.parametrize("case,code", [
    (dict(N=16384, t=1146881, q=[1073643521, 1073479681], P=1073479681), -2),   # repeated modulus
    (dict(N=16384, t=1146881, q=[1073643521, 1073479683], P=1071415297), -2),   # not prime
    (dict(N=16384, t=12289, q=[1073643521], P=1071415297), -2),                 # t != 1 mod 2N
    (dict(N=4096, t=65537, q=[1073692673, 1073668097, 1073651713], P=1073643521), -3),  # over the cap
    (dict(N=3000, t=65537, q=[1073692673], P=1073668097), -2),                  # N not a power of two
    # a second special prime: repeated, below 2^29, and over the cap with it
    (dict(N=16384, t=1146881, q=[1073643521, 1073479681], P=1073184769, P2=1073184769), -2),
    (dict(N=4096, t=65537, q=[1073692673], P=1073668097, P2=40961), -2),
    (dict(N=4096, t=65537, q=[1073692673, 1073668097], P=1073651713, P2=1073643521), -3),
])
def test_parameter_validation_errors(lib, case, code):
    q = (ctypes.c_uint32 * len(case["q"]))(*case["q"])
    p = _Params(case["N"], case["t"], len(case["q"]), q, case["P"], 0, case.get("P2", 0))
    h = ctypes.c_void_p()
    lib.lola_ctx_create.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    lib.lola_last_error.restype = ctypes.c_char_p
    assert lib.lola_ctx_create(ctypes.byref(p), 0, ctypes.byref(h)) == code
    assert lib.lola_last_error()
