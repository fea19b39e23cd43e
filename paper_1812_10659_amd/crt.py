"""Exact integer outputs: one network run under several plaintext moduli.

Each plaintext modulus t_i has its own context (the same ciphertext primes),
compiled plan and client keys; a request is encrypted, evaluated and
decrypted once per modulus, and the outputs mod t_i are combined on the device
by `lola_crt_combine` into exact signed integers (Sec. 4.4 runs its CIFAR
network under three plaintext moduli the same way).  Argument marshalling
only: encryption, evaluation, decryption, decoding and the combination all run
in the library.
"""
from __future__ import annotations

import ctypes
from typing import List, Sequence

import numpy as np
import torch

from . import lola, networks
from . import workloads as wl


def _sig():
    L = lola._plan_sig()
    if not getattr(L, "_crt_sig", False):
        f = L.lola_crt_combine
        f.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32,
                      ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]
        f.restype = ctypes.c_int32
        L._crt_sig = True
    return L


def words_for(moduli: Sequence[int]) -> int:
    """64-bit words that hold every signed value in [-M/2, M/2)."""
    return (int(np.prod([int(t) for t in moduli], dtype=object)).bit_length() + 63) // 64


def crt_combine(residues: Sequence[torch.Tensor], moduli: Sequence[int], words: int | None = None) -> torch.Tensor:
    """residues: k device int64 tensors of n values, tensor i mod moduli[i].
    Returns [n][words] int64 (device), little-endian two's complement."""
    k = len(moduli)
    n = residues[0].numel()
    w = words_for(moduli) if words is None else words
    out = torch.empty((n, w), dtype=torch.int64, device=residues[0].device)
    ptrs = (ctypes.c_void_p * k)(*[r.data_ptr() for r in residues])
    mods = (ctypes.c_uint32 * k)(*[int(t) for t in moduli])
    lola._check(_sig().lola_crt_combine(ptrs, mods, k, n, out.data_ptr(), w, lola._stream()))
    return out


def words_to_ints(words: np.ndarray) -> List[int]:
    """[n][w] little-endian two's complement words -> Python integers."""
    a = np.asarray(words, dtype=np.int64)
    bits = 64 * a.shape[1]
    out = []
    for row in a:
        v = 0
        for j, x in enumerate(row):
            v |= (int(x) & 0xFFFFFFFFFFFFFFFF) << (64 * j)
        out.append(v - (1 << bits) if v >> (bits - 1) else v)
    return out


class CrtNetwork:
    """A layer list compiled once per plaintext modulus of `params`."""

    def __init__(self, params: Sequence[wl.ParamSet], layers, device: int = 0):
        self.params = list(params)
        self.moduli = [p.t for p in self.params]
        self.ctxs = [lola.Context(p, device) for p in self.params]
        self.plans = [lola.Plan(p, layers) for p in self.params]
        for c, pl in zip(self.ctxs, self.plans):
            pl.load(c)
        self.words = words_for(self.moduli)

    def keygen(self, seed: int) -> list:
        """One key set per modulus (secret, public, relinearisation, Galois)."""
        keys = []
        for c, pl in zip(self.ctxs, self.plans):
            sk = c.keygen_secret(seed)
            keys.append(dict(sk=sk, pk=c.keygen_public(seed, sk), rlk=c.keygen_switch(seed, sk, 0),
                             gks=[c.keygen_switch(seed, sk, g) for g in pl.galois()]))
        return keys

    def request(self, keys: list, values: np.ndarray, seed: int) -> list:
        """Encrypted inputs and empty outputs of one request, per modulus."""
        reqs = []
        for c, pl, k in zip(self.ctxs, self.plans, keys):
            msgs = networks.pack_inputs(pl.input_map(), values)
            ins = [c.encrypt(k["pk"], c.encode(m), seed, i) for i, m in enumerate(msgs)]
            reqs.append(dict(rlk=k["rlk"], gks=k["gks"], inputs=ins,
                             outputs=[c.empty_ct() for _ in range(pl.info["n_outputs"])]))
        return reqs

    def evaluate(self, requests: list) -> None:
        """requests: per request, the list returned by `request`."""
        for i, (c, pl) in enumerate(zip(self.ctxs, self.plans)):
            pl.evaluate(c, [r[i] for r in requests])

    def integers(self, keys: list, request: list) -> List[int]:
        """Decrypts one evaluated request under every modulus and returns its
        outputs as exact integers."""
        res = []
        for i, c in enumerate(self.ctxs):
            outs = request[i]["outputs"]
            slots = torch.empty((len(outs), c.N), dtype=torch.int64, device=c.device)
            for j, o in enumerate(outs):
                c.decode_dev(c.decrypt(keys[i]["sk"], o), out=slots[j])
            res.append(slots.reshape(-1))
        omap = self.plans[0].output_map().reshape(-1)
        sel = np.nonzero(omap >= 0)[0]
        words = crt_combine(res, self.moduli, self.words).cpu().numpy()[sel]
        out = [0] * (int(omap.max()) + 1)
        for v, idx in zip(words_to_ints(words), omap[sel]):
            out[int(idx)] = v
        return out
