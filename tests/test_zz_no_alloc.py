"""The rotation that allocates nothing (lola_rotate_noalloc, scratch in a
fixed device array) against lola_rotate on the same inputs, word for word,
through the C ABI: calls in a row, each smaller than the one before (the
largest shape the fixed array holds, twelve primes with two special primes;
then seven primes with two-prime digits, with one prime per digit, and a
smaller ring), so that each runs over the previous call's leftovers in the
shared array."""
import ctypes

import numpy as np
import pytest

from paper_1812_10659_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _noalloc():
    from paper_1812_10659_amd import lola
    f = lola.lib().lola_rotate_noalloc
    vp = ctypes.c_void_p
    f.argtypes = [vp, vp, ctypes.c_uint32, vp, vp, vp]
    f.restype = ctypes.c_int32
    return f


def test_rotate_noalloc_equals_rotate_second_call_smaller():
    import torch
    from paper_1812_10659_amd import lola
    f = _noalloc()
    # (parameter set, step): the second call is the smaller one
    for k, (pname, step) in enumerate([("l12_n16384_k2", 7), ("mnist_n16384_k2", 5), ("mnist_n16384", 3),
                                       ("n4096_3q", "row_swap")]):
        p = wl.PARAMS[pname]
        print(f"[gpu-noalloc] call {k}: {pname} step {step}", flush=True)
        ctx = lola.Context(p)
        seed = 4242 + k
        sk = ctx.keygen_secret(seed)
        pk = ctx.keygen_public(seed, sk)
        g = lola.galois_element(p.N, step)
        gk = ctx.keygen_switch(seed, sk, g)
        v = wl.rng(seed, 1).integers(0, p.t, p.N)
        ct = ctx.encrypt(pk, ctx.encode(v), seed, 0)
        ref = ctx.rotate(gk, g, ct)
        out = ctx.empty_ct()
        out.fill_(-1)
        torch.cuda.synchronize()
        lola._check(f(ctx.h, gk.data_ptr(), g, ct.data_ptr(), out.data_ptr(),
                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"call {k} ({pname})"
        # and it decrypts to the rotated slots
        got = ctx.decode(ctx.decrypt(sk, out))
        from oracle import network as nw
        assert np.array_equal(got, nw.rotate_slots(np.asarray(v) % p.t, step))
        ctx.close()


def test_rotate_noalloc_rejects_bad_arguments():
    import torch
    from paper_1812_10659_amd import lola
    f = _noalloc()
    p = wl.PARAMS["n4096_3q"]
    ctx = lola.Context(p)
    ct, out = ctx.empty_ct(), ctx.empty_ct()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    key = ctx.empty(ctx.dnum, 2, p.L + ctx.K, p.N)
    code = {v: k for k, v in lola.E_CODES.items()}
    assert f(ctx.h, None, 3, ct.data_ptr(), out.data_ptr(), s) == code["E_NOKEY"]
    assert f(ctx.h, key.data_ptr(), 4, ct.data_ptr(), out.data_ptr(), s) == code["E_INVAL"]
    assert f(ctx.h, key.data_ptr(), 3, ct.data_ptr(), ct.data_ptr(), s) == code["E_INVAL"]
    ctx.close()
