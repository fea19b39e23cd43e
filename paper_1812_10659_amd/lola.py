"""Python binding of liblola (include/lola.h): argument marshalling only.

Every operation runs in the HIP library; this module converts torch device
tensors to pointers, passes the current HIP stream, and raises LolaError on a
non-zero return code.  torch provides device memory and streams.  Buffers are
int32 tensors holding the library's uint32 words.

The library must be built (paper_1812_10659_amd/build_lib.py, or
__graft_entry__.build()); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblola.so")

ROW_SWAP = 0x7FFFFFFF

E_CODES = {0: "OK", -1: "E_INVAL", -2: "E_PARAMS", -3: "E_INSECURE", -4: "E_SHAPE", -5: "E_NOKEY",
           -6: "E_NOMEM", -7: "E_DEVICE", -8: "E_UNSUPPORTED"}


class LolaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{E_CODES.get(code, code)}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("t", ctypes.c_uint32), ("L", ctypes.c_uint32),
                ("q", ctypes.POINTER(ctypes.c_uint32)), ("P", ctypes.c_uint32),
                ("allow_insecure", ctypes.c_int), ("P2", ctypes.c_uint32)]


class _Info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("L", ctypes.c_uint32), ("t", ctypes.c_uint32),
                ("n_aux", ctypes.c_uint32), ("ct_words", ctypes.c_uint64),
                ("poly_words", ctypes.c_uint64), ("sk_words", ctypes.c_uint64),
                ("ksk_words", ctypes.c_uint64), ("scratch_bytes", ctypes.c_uint64),
                ("K", ctypes.c_uint32), ("dnum", ctypes.c_uint32)]


class KsDesc(ctypes.Structure):
    _fields_ = [("in_dev", ctypes.c_void_p), ("key_dev", ctypes.c_void_p), ("out_dev", ctypes.c_void_p),
                ("galois", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


_lib = None


class NttVariant(ctypes.Structure):
    _fields_ = [("split", ctypes.c_uint32), ("limbs_per_wg", ctypes.c_uint32), ("ms", ctypes.c_float)]


class KsVariant(ctypes.Structure):
    _fields_ = [("stage", ctypes.c_uint32), ("index", ctypes.c_uint32), ("split", ctypes.c_uint32),
                ("padded", ctypes.c_uint32), ("ms", ctypes.c_float)]


KS_STAGES = ("digits", "inner", "moddown")


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1812_10659_amd/build_lib.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32, i64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64
        sig = {
            "lola_ctx_create": [ctypes.POINTER(_Params), i32, ctypes.POINTER(vp)],
            "lola_ctx_destroy": [vp],
            "lola_ctx_info": [vp, ctypes.POINTER(_Info)],
            "lola_reserve": [vp, u32],
            "lola_galois_element": [u32, ctypes.c_int32],
            "lola_keygen_secret": [vp, u64, vp, vp],
            "lola_keygen_public": [vp, u64, vp, vp, vp],
            "lola_keygen_switch": [vp, u64, vp, u32, vp, vp],
            "lola_encode": [vp, vp, vp, vp],
            "lola_decode": [vp, vp, vp, vp],
            "lola_encode_batch": [vp, vp, u32, vp, vp],
            "lola_decode_batch": [vp, vp, u32, vp, vp],
            "lola_plain_mul_form": [vp, vp, vp, vp],
            "lola_plain_add_form": [vp, vp, vp, vp],
            "lola_encrypt": [vp, vp, vp, u64, u32, vp, vp],
            "lola_decrypt": [vp, vp, vp, u32, vp, vp],
            "lola_encrypt_batch": [vp, vp, vp, u32, u64, u32, vp, vp],
            "lola_decrypt_batch": [vp, vp, vp, u32, u32, vp, vp],
            "lola_add": [vp, vp, vp, u32, vp, vp],
            "lola_add_plain": [vp, vp, vp, vp, vp],
            "lola_mul_plain": [vp, vp, vp, vp, vp],
            "lola_mul_scalar": [vp, vp, i64, vp, vp],
            "lola_mul": [vp, vp, vp, vp, vp],
            "lola_relin": [vp, vp, vp, vp, vp],
            "lola_rotate": [vp, vp, u32, vp, vp, vp],
            "lola_rotate_hoisted": [vp, vp, u32, ctypes.POINTER(u32), ctypes.POINTER(vp), ctypes.POINTER(vp), vp],
            "lola_keyswitch_batch": [vp, ctypes.POINTER(KsDesc), u32, vp],
            "lola_to_coeff": [vp, vp, u32, vp, vp],
            "lola_from_coeff": [vp, vp, u32, vp, vp],
            "lola_export_sk": [vp, vp, vp, vp],
            "lola_export_pk": [vp, vp, vp, vp],
            "lola_export_ksk": [vp, vp, vp, vp],
            "lola_ntt_limbs": [vp, vp, vp, u32, ctypes.POINTER(u32), i32, vp],
            "lola_ntt_variants": [vp, ctypes.POINTER(NttVariant), u32, ctypes.POINTER(u32)],
            "lola_ntt_get_variant": [vp, ctypes.POINTER(u32)],
            "lola_ntt_set_variant": [vp, u32],
            "lola_ntt_autotune": [vp, u32, u32, ctypes.POINTER(NttVariant), u32, ctypes.POINTER(u32), vp],
            "lola_ks_variants": [vp, u32, ctypes.POINTER(KsVariant), u32, ctypes.POINTER(u32)],
            "lola_ks_get_variant": [vp, u32, ctypes.POINTER(u32)],
            "lola_ks_set_variant": [vp, u32, u32],
            "lola_ks_autotune": [vp, u32, u32, ctypes.POINTER(KsVariant), u32, ctypes.POINTER(u32), vp],
            "lola_set_key_words": [vp, ctypes.POINTER(u32)],
            "lola_strerror": [i32],
            "lola_last_error": [],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.lola_ctx_destroy.restype = None
        L.lola_galois_element.restype = u32
        L.lola_strerror.restype = ctypes.c_char_p
        L.lola_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        raise LolaError(rc, lib().lola_last_error().decode())


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def galois_element(N: int, step) -> int:
    return int(lib().lola_galois_element(N, ROW_SWAP if step == "row_swap" else int(step)))


class Context:
    """lola_ctx for one parameter set (N, t, q, P and, for digits of two
    primes, P2) on one device."""

    def __init__(self, params, device: int = 0):
        self.params = params
        self.device = torch.device("cuda", device)
        p, q = _params_struct(params)
        h = ctypes.c_void_p()
        _check(lib().lola_ctx_create(ctypes.byref(p), device, ctypes.byref(h)))
        self.h = h
        info = _Info()
        _check(lib().lola_ctx_info(self.h, ctypes.byref(info)))
        self.N, self.L, self.t, self.n_aux = info.N, info.L, info.t, info.n_aux
        self.K, self.dnum = info.K, info.dnum
        self.ksk_words = info.ksk_words

    def close(self):
        if getattr(self, "h", None):
            lib().lola_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 (interpreter shutdown)
            pass

    # ---- buffers
    def empty(self, *shape) -> torch.Tensor:
        return torch.empty(*shape, dtype=torch.int32, device=self.device)

    def empty_ct(self, size: int = 2) -> torch.Tensor:
        return self.empty(size, self.L, self.N)

    def reserve(self, n_ct: int) -> None:
        _check(lib().lola_reserve(self.h, n_ct))

    # ---- keys
    def set_key_words(self, words) -> None:
        """ChaCha20 key words 2..7 (six 32-bit values) for every later key
        generation and encryption; None = zeros (the 64-bit seed alone)."""
        arr = None if words is None else (ctypes.c_uint32 * 6)(*[int(w) & 0xFFFFFFFF for w in words])
        _check(lib().lola_set_key_words(self.h, arr))

    def keygen_secret(self, seed: int) -> torch.Tensor:
        sk = self.empty(self.L + self.K, self.N)
        _check(lib().lola_keygen_secret(self.h, seed, _p(sk), _stream()))
        return sk

    def keygen_public(self, seed: int, sk: torch.Tensor) -> torch.Tensor:
        pk = self.empty(2, self.L, self.N)
        _check(lib().lola_keygen_public(self.h, seed, _p(sk), _p(pk), _stream()))
        return pk

    def keygen_switch(self, seed: int, sk: torch.Tensor, galois: int) -> torch.Tensor:
        k = self.empty(self.dnum, 2, self.L + self.K, self.N)
        _check(lib().lola_keygen_switch(self.h, seed, _p(sk), galois, _p(k), _stream()))
        return k

    # ---- plaintexts
    def encode(self, slots) -> torch.Tensor:
        s = torch.as_tensor(np.asarray(slots, dtype=np.int64)).to(self.device)
        pt = self.empty(self.N)
        _check(lib().lola_encode(self.h, _p(s), _p(pt), _stream()))
        return pt

    def decode(self, pt: torch.Tensor) -> np.ndarray:
        return self.decode_dev(pt).cpu().numpy()

    def decode_dev(self, pt: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Slots of a plaintext as a device int64 tensor of N values in [0, t)."""
        s = torch.empty(self.N, dtype=torch.int64, device=self.device) if out is None else out
        _check(lib().lola_decode(self.h, _p(pt), _p(s), _stream()))
        return s

    def encode_batch(self, slots, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """slots: [n][N] integers (host array or device int64 tensor), one host
        to device copy for all; returns [n][N] plaintexts."""
        s = slots if isinstance(slots, torch.Tensor) else torch.as_tensor(np.asarray(slots, dtype=np.int64))
        s = s.to(device=self.device, dtype=torch.int64).contiguous()
        n = s.shape[0]
        pt = self.empty(n, self.N) if out is None else out
        _check(lib().lola_encode_batch(self.h, _p(s), n, _p(pt), _stream()))
        return pt

    def decode_batch(self, pts: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """[n][N] plaintexts -> [n][N] device int64 slots in [0, t)."""
        n = pts.shape[0]
        s = torch.empty((n, self.N), dtype=torch.int64, device=self.device) if out is None else out
        _check(lib().lola_decode_batch(self.h, _p(pts), n, _p(s), _stream()))
        return s

    def plain_mul_form(self, pt: torch.Tensor) -> torch.Tensor:
        out = self.empty(self.L, self.N)
        _check(lib().lola_plain_mul_form(self.h, _p(pt), _p(out), _stream()))
        return out

    def plain_add_form(self, pt: torch.Tensor) -> torch.Tensor:
        out = self.empty(self.L, self.N)
        _check(lib().lola_plain_add_form(self.h, _p(pt), _p(out), _stream()))
        return out

    # ---- encrypt / decrypt
    def encrypt(self, pk, pt, seed: int, nonce: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        ct = self.empty_ct() if out is None else out
        _check(lib().lola_encrypt(self.h, _p(pk), _p(pt), seed, nonce, _p(ct), _stream()))
        return ct

    def encrypt_batch(self, pk, pts: torch.Tensor, seed: int, nonce0: int,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """[n][N] plaintexts -> [n][2][L][N] ciphertexts, message i with
        object id nonce0 + i."""
        n = pts.shape[0]
        ct = self.empty(n, 2, self.L, self.N) if out is None else out
        _check(lib().lola_encrypt_batch(self.h, _p(pk), _p(pts), n, seed, nonce0, _p(ct), _stream()))
        return ct

    def decrypt_batch(self, sk, cts: torch.Tensor) -> torch.Tensor:
        """[n][size][L][N] ciphertexts -> [n][N] plaintexts."""
        n, size = cts.shape[0], cts.shape[1]
        pt = self.empty(n, self.N)
        _check(lib().lola_decrypt_batch(self.h, _p(sk), _p(cts), n, size, _p(pt), _stream()))
        return pt

    def decrypt(self, sk, ct) -> torch.Tensor:
        pt = self.empty(self.N)
        _check(lib().lola_decrypt(self.h, _p(sk), _p(ct), ct.shape[0], _p(pt), _stream()))
        return pt

    # ---- operations
    def add(self, a, b, out=None):
        out = self.empty_ct(a.shape[0]) if out is None else out
        _check(lib().lola_add(self.h, _p(a), _p(b), a.shape[0], _p(out), _stream()))
        return out

    def add_plain(self, ct, pta, out=None):
        out = self.empty_ct() if out is None else out
        _check(lib().lola_add_plain(self.h, _p(ct), _p(pta), _p(out), _stream()))
        return out

    def mul_plain(self, ct, ptm, out=None):
        out = self.empty_ct() if out is None else out
        _check(lib().lola_mul_plain(self.h, _p(ct), _p(ptm), _p(out), _stream()))
        return out

    def mul_scalar(self, ct, w: int, out=None):
        out = self.empty_ct() if out is None else out
        _check(lib().lola_mul_scalar(self.h, _p(ct), int(w), _p(out), _stream()))
        return out

    def mul(self, a, b):
        out = self.empty_ct(3)
        _check(lib().lola_mul(self.h, _p(a), _p(b), _p(out), _stream()))
        return out

    def relin(self, rlk, ct3):
        out = self.empty_ct()
        _check(lib().lola_relin(self.h, _p(rlk), _p(ct3), _p(out), _stream()))
        return out

    def rotate(self, gk, galois: int, ct):
        out = self.empty_ct()
        _check(lib().lola_rotate(self.h, _p(gk), galois, _p(ct), _p(out), _stream()))
        return out

    def rotate_hoisted(self, ct: torch.Tensor, galois: Sequence[int], keys: Sequence[torch.Tensor]) -> list:
        """Rotations of one ciphertext by each Galois element, sharing its
        decomposition (lola_rotate_hoisted)."""
        n = len(galois)
        outs = [self.empty_ct() for _ in range(n)]
        g = (ctypes.c_uint32 * n)(*[int(x) for x in galois])
        k = (ctypes.c_void_p * n)(*[t.data_ptr() for t in keys])
        o = (ctypes.c_void_p * n)(*[t.data_ptr() for t in outs])
        _check(lib().lola_rotate_hoisted(self.h, ct.data_ptr(), n, g, k, o, _stream()))
        return outs

    def keyswitch_batch(self, items: Sequence) -> list:
        """items: (input ct, key, galois) with galois 0 for relinearisation."""
        outs = [self.empty_ct() for _ in items]
        arr = (KsDesc * len(items))()
        for k, (ct, key, g) in enumerate(items):
            arr[k] = KsDesc(ct.data_ptr(), key.data_ptr(), outs[k].data_ptr(), g, 0)
        _check(lib().lola_keyswitch_batch(self.h, arr, len(items), _stream()))
        return outs

    # ---- canonical forms
    def to_coeff(self, x: torch.Tensor) -> torch.Tensor:
        n = x.numel() // (self.L * self.N)
        out = torch.empty_like(x)
        _check(lib().lola_to_coeff(self.h, _p(x), n, _p(out), _stream()))
        return out

    def from_coeff(self, x: torch.Tensor) -> torch.Tensor:
        n = x.numel() // (self.L * self.N)
        out = torch.empty_like(x)
        _check(lib().lola_from_coeff(self.h, _p(x), n, _p(out), _stream()))
        return out

    def export_sk(self, sk):
        out = torch.empty_like(sk)
        _check(lib().lola_export_sk(self.h, _p(sk), _p(out), _stream()))
        return out

    def export_pk(self, pk):
        out = torch.empty_like(pk)
        _check(lib().lola_export_pk(self.h, _p(pk), _p(out), _stream()))
        return out

    def export_ksk(self, k):
        out = torch.empty_like(k)
        _check(lib().lola_export_ksk(self.h, _p(k), _p(out), _stream()))
        return out

    def ntt_variants(self) -> list:
        """[(split, limbs_per_wg)] of the batched NTT variants compiled for this N."""
        n = ctypes.c_uint32()
        _check(lib().lola_ntt_variants(self.h, None, 0, ctypes.byref(n)))
        arr = (NttVariant * n.value)()
        _check(lib().lola_ntt_variants(self.h, arr, n.value, ctypes.byref(n)))
        return [(v.split, v.limbs_per_wg) for v in arr]

    def ntt_variant(self) -> int:
        k = ctypes.c_uint32()
        _check(lib().lola_ntt_get_variant(self.h, ctypes.byref(k)))
        return k.value

    def ntt_set_variant(self, index: int) -> None:
        _check(lib().lola_ntt_set_variant(self.h, int(index)))

    def ks_variants(self, stage: int) -> list:
        """[(split, padded)] of a key-switch stage's variants (0 digits, 1
        inner, 2 mod-down) compiled for this N."""
        n = ctypes.c_uint32()
        _check(lib().lola_ks_variants(self.h, int(stage), None, 0, ctypes.byref(n)))
        arr = (KsVariant * n.value)()
        _check(lib().lola_ks_variants(self.h, int(stage), arr, n.value, ctypes.byref(n)))
        return [(v.split, v.padded) for v in arr]

    def ks_variant(self, stage: int) -> int:
        k = ctypes.c_uint32()
        _check(lib().lola_ks_get_variant(self.h, int(stage), ctypes.byref(k)))
        return k.value

    def ks_set_variant(self, stage: int, index: int) -> None:
        _check(lib().lola_ks_set_variant(self.h, int(stage), int(index)))

    def ks_autotune(self, n_jobs: int = 128, reps: int = 10):
        """Times every key-switch stage variant (a batch of n_jobs rotations,
        each variant's words checked against the default first), keeps the
        fastest per stage; returns (chosen [3], [(stage, index, split,
        padded, ms)])."""
        n = sum(len(self.ks_variants(st)) for st in range(3))
        arr = (KsVariant * n)()
        ch = (ctypes.c_uint32 * 3)()
        _check(lib().lola_ks_autotune(self.h, int(n_jobs), int(reps), arr, n, ch, _stream()))
        return list(ch), [(v.stage, v.index, v.split, v.padded, float(v.ms)) for v in arr]

    def ntt_autotune(self, n_limbs: int = 512, reps: int = 5):
        """Times every batched NTT variant (forward + inverse of n_limbs limbs),
        keeps the fastest; returns (chosen index, [(split, limbs_per_wg, ms)])."""
        n = len(self.ntt_variants())
        arr = (NttVariant * n)()
        k = ctypes.c_uint32()
        _check(lib().lola_ntt_autotune(self.h, int(n_limbs), int(reps), arr, n, ctypes.byref(k), _stream()))
        return k.value, [(v.split, v.limbs_per_wg, float(v.ms)) for v in arr]

    def ntt_limbs(self, x: torch.Tensor, prime_idx: Iterable[int], inverse: bool = False) -> torch.Tensor:
        """prime_idx: one prime index per limb; a uint32 numpy array passes
        through without conversion (a list is converted on every call)."""
        idx = np.ascontiguousarray(np.asarray(prime_idx, dtype=np.uint32))
        out = torch.empty_like(x)
        _check(lib().lola_ntt_limbs(self.h, _p(x), _p(out), idx.size,
                                    idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), int(inverse), _stream()))
        return out


def to_numpy_u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def from_numpy_u32(a: np.ndarray, device) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(device)


# ------------------------------------------------------------- plans -----
LAYER_CONV2D, LAYER_DENSE, LAYER_SQUARE, LAYER_CONV2D_DENSE_INPUT = 1, 2, 3, 4


class Layer(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("in_h", ctypes.c_int32), ("in_w", ctypes.c_int32),
                ("k", ctypes.c_int32), ("stride", ctypes.c_int32), ("maps", ctypes.c_int32),
                ("in_dim", ctypes.c_int32), ("out_dim", ctypes.c_int32),
                ("weight", ctypes.POINTER(ctypes.c_int64)), ("bias", ctypes.POINTER(ctypes.c_int64))]


class _PlanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "n_inputs", "n_outputs", "n_ops", "n_consts", "n_galois", "n_waves", "queries",
        "n_rotations", "n_mul_plain", "n_mul_scalar", "n_square", "n_add_plain", "n_add", "n_phys_regs",
        "recipe")] + [("predicted_us", ctypes.c_float), ("predicted_latency_us", ctypes.c_float),
                      ("sums", ctypes.c_uint32)]


class _CompileOptions(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_int32), ("recipe", ctypes.c_int32), ("sums", ctypes.c_int32)]


OBJECTIVE_THROUGHPUT, OBJECTIVE_LATENCY = 0, 1
RECIPE_AUTO, RECIPE_DENSE_ROW_MAJOR, RECIPE_STACKED_ROW_MAJOR, RECIPE_FIXED = 0, 1, 2, 3
RECIPE_FULL_REDUCTION, RECIPE_SHARED_REDUCTION = 4, 5
RECIPE_DENSE_CHAIN, RECIPE_SPARSE_COLUMN_MAJOR = 6, 7
SUMS_AUTO, SUMS_SEQUENTIAL, SUMS_HOISTED = 0, 1, 2


class Request(ctypes.Structure):
    _fields_ = [("rlk_dev", ctypes.c_void_p), ("gk_dev", ctypes.POINTER(ctypes.c_void_p)),
                ("in_dev", ctypes.POINTER(ctypes.c_void_p)), ("out_dev", ctypes.POINTER(ctypes.c_void_p))]


def conv2d(weight, bias, in_hw: int, stride: int, dense_input: bool = False) -> dict:
    """weight: [maps][k][k] or [maps][channels][k][k].  dense_input: the
    client sends the padded image as one dense message (row by row) instead of
    the k*k convolution-representation messages."""
    w = np.ascontiguousarray(weight, dtype=np.int64)
    kind = LAYER_CONV2D_DENSE_INPUT if dense_input else LAYER_CONV2D
    channels = w.shape[1] if w.ndim == 4 else 0
    return dict(kind=kind, in_h=in_hw, in_w=in_hw, k=w.shape[-1], stride=stride, maps=w.shape[0], in_dim=channels,
                weight=w, bias=None if bias is None else np.ascontiguousarray(bias, dtype=np.int64))


def dense(weight, bias=None) -> dict:
    w = np.ascontiguousarray(weight, dtype=np.int64)
    return dict(kind=LAYER_DENSE, in_dim=w.shape[1], out_dim=w.shape[0], weight=w,
                bias=None if bias is None else np.ascontiguousarray(bias, dtype=np.int64))


def square() -> dict:
    return dict(kind=LAYER_SQUARE)


def _params_struct(params):
    q = (ctypes.c_uint32 * len(params.q))(*params.q)
    return _Params(params.N, params.t, len(params.q), q, params.P, int(getattr(params, "insecure_ok", False)),
                   int(getattr(params, "P2", 0))), q


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("total_ms", ctypes.c_double), ("launches", ctypes.c_uint64),
                ("units", ctypes.c_uint64), ("alg_bytes", ctypes.c_double), ("alg_ops", ctypes.c_double)]


def _plan_sig():
    L = lib()
    if getattr(L, "_plan_sig_done", False):
        return L
    vp, u32 = ctypes.c_void_p, ctypes.c_uint32
    sig = {
        "lola_compile": [ctypes.POINTER(_Params), ctypes.POINTER(Layer), u32, ctypes.POINTER(vp)],
        "lola_compile_ex": [ctypes.POINTER(_Params), ctypes.POINTER(Layer), u32, ctypes.POINTER(_CompileOptions),
                            ctypes.POINTER(vp)],
        "lola_plan_get_info": [vp, ctypes.POINTER(_PlanInfo)],
        "lola_plan_galois": [vp, ctypes.POINTER(u32)],
        "lola_plan_input_map": [vp, ctypes.POINTER(ctypes.c_int32)],
        "lola_plan_output_map": [vp, ctypes.POINTER(ctypes.c_int32)],
        "lola_plan_dump": [vp, ctypes.c_char_p, ctypes.c_size_t],
        "lola_plan_const": [vp, u32, ctypes.POINTER(ctypes.c_int64)],
        "lola_plan_load": [vp, vp, vp],
        "lola_evaluate": [vp, vp, ctypes.POINTER(Request), u32, vp],
        "lola_evaluate_graph": [vp, vp, ctypes.POINTER(Request), u32, vp],
        "lola_plan_set_lanes": [vp, u32],
        "lola_timing_enable": [vp, ctypes.c_int],
        "lola_kernel_timing": [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64),
                               ctypes.POINTER(ctypes.c_uint64)],
        "lola_kernel_stats": [vp, ctypes.POINTER(KernelStat), u32, ctypes.POINTER(u32)],
        "lola_plan_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    L.lola_plan_destroy.restype = None
    L._plan_sig_done = True
    return L


class Plan:
    """lola_plan: a layer list compiled for a parameter set (host logic)."""

    def __init__(self, params, layers, objective: int = OBJECTIVE_THROUGHPUT, recipe: int = RECIPE_AUTO,
                 sums: int = SUMS_AUTO):
        L = _plan_sig()
        arr = (Layer * len(layers))()
        self._keep = []
        for k, d in enumerate(layers):
            ly = Layer()
            for f in ("kind", "in_h", "in_w", "k", "stride", "maps", "in_dim", "out_dim"):
                setattr(ly, f, int(d.get(f, 0)))
            for f in ("weight", "bias"):
                a = d.get(f)
                if a is not None:
                    self._keep.append(a)
                    setattr(ly, f, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
            arr[k] = ly
        ps, self._q = _params_struct(params)
        h = ctypes.c_void_p()
        opts = _CompileOptions(int(objective), int(recipe), int(sums))
        _check(L.lola_compile_ex(ctypes.byref(ps), arr, len(layers), ctypes.byref(opts), ctypes.byref(h)))
        self.h = h
        self._keep = []
        self.N = params.N
        inf = _PlanInfo()
        _check(L.lola_plan_get_info(self.h, ctypes.byref(inf)))
        self.info = {f: getattr(inf, f) for f, _ in _PlanInfo._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().lola_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def galois(self) -> list:
        n = self.info["n_galois"]
        a = (ctypes.c_uint32 * max(n, 1))()
        _check(lib().lola_plan_galois(self.h, a))
        return [int(a[i]) for i in range(n)]

    def input_map(self) -> np.ndarray:
        a = np.empty(self.info["n_inputs"] * self.N, np.int32)
        _check(lib().lola_plan_input_map(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return a.reshape(self.info["n_inputs"], self.N)

    def output_map(self) -> np.ndarray:
        a = np.empty(self.info["n_outputs"] * self.N, np.int32)
        _check(lib().lola_plan_output_map(self.h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return a.reshape(self.info["n_outputs"], self.N)

    def dump(self) -> str:
        need = lib().lola_plan_dump(self.h, None, 0)
        buf = ctypes.create_string_buffer(need)
        _check(lib().lola_plan_dump(self.h, buf, need))
        return buf.value.decode()

    def const(self, cid: int) -> np.ndarray:
        a = np.empty(self.N, np.int64)
        _check(lib().lola_plan_const(self.h, cid, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return a

    def load(self, ctx: "Context") -> None:
        _check(lib().lola_plan_load(ctx.h, self.h, _stream()))

    def set_lanes(self, max_lanes: int) -> None:
        """1: every batch on the caller's stream; 2 (default): batches of 16 or
        more requests as two lanes on two streams."""
        _check(_plan_sig().lola_plan_set_lanes(self.h, int(max_lanes)))

    def evaluate(self, ctx: "Context", requests, graph: bool = False, stream=None) -> None:
        """requests: list of dict(rlk=tensor, gks=[tensor per galois()], inputs=[...], outputs=[...])."""
        n = len(requests)
        arr = (Request * n)()
        keep = []
        for k, r in enumerate(requests):
            gk = (ctypes.c_void_p * max(len(r["gks"]), 1))(*[t.data_ptr() for t in r["gks"]])
            ins = (ctypes.c_void_p * len(r["inputs"]))(*[t.data_ptr() for t in r["inputs"]])
            outs = (ctypes.c_void_p * len(r["outputs"]))(*[t.data_ptr() for t in r["outputs"]])
            keep += [gk, ins, outs]
            arr[k] = Request(r["rlk"].data_ptr() if r.get("rlk") is not None else None,
                             ctypes.cast(gk, ctypes.POINTER(ctypes.c_void_p)),
                             ctypes.cast(ins, ctypes.POINTER(ctypes.c_void_p)),
                             ctypes.cast(outs, ctypes.POINTER(ctypes.c_void_p)))
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream()
        f = lib().lola_evaluate_graph if graph else lib().lola_evaluate
        _check(f(ctx.h, self.h, arr, n, s))


def timing_enable(ctx: "Context", on: bool) -> None:
    _check(_plan_sig().lola_timing_enable(ctx.h, int(on)))


def kernel_timing(ctx: "Context"):
    """(total ms, launches, jobs) of the key-switch inner kernel since the last read."""
    ms, n, j = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(_plan_sig().lola_kernel_timing(ctx.h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(j)))
    return ms.value, n.value, j.value


def kernel_stats(ctx: "Context") -> dict:
    """Per timed kernel since the last read: {name: dict(ms, launches, units,
    alg_bytes, alg_ops)} (the library's event times and algorithmic charges)."""
    L = _plan_sig()
    cap = 64
    arr = (KernelStat * cap)()
    n = ctypes.c_uint32()
    _check(L.lola_kernel_stats(ctx.h, arr, cap, ctypes.byref(n)))
    return {arr[i].name.decode(): dict(ms=arr[i].total_ms, launches=int(arr[i].launches), units=int(arr[i].units),
                                       alg_bytes=arr[i].alg_bytes, alg_ops=arr[i].alg_ops)
            for i in range(n.value)}


def valu_probe(op: int, iters: int = 2000) -> float:
    """Achieved lane-instructions per second of one 32-bit VALU instruction
    kind (0 v_mul_lo_u32, 1 v_mul_hi_u32, 2 v_add_u32) over the whole GPU."""
    L = lib()
    f = L.lola_valu_probe
    f.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double),
                  ctypes.c_void_p]
    f.restype = ctypes.c_int32
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    buf = torch.empty(2048 * cus, dtype=torch.int32, device="cuda")
    rate = ctypes.c_double()
    _check(f(int(op), int(iters), ctypes.c_void_p(buf.data_ptr()), buf.numel(), ctypes.byref(rate), _stream()))
    return rate.value
