"""GPU edge cases: empty and ragged batches, error codes of the C ABI, and
determinism.  Every error case here is rejected by the library's host-side
checks before anything is launched."""
import ctypes

import numpy as np
import pytest

from oracle import bfv
from paper_1812_10659_amd import workloads as wl

pytestmark = pytest.mark.gpu

SEED = 0x5EED_0002


# one prime per key-switching digit, and digits of two primes with two
# special primes
@pytest.fixture(scope="module", params=["toy1024", "toy1024_k2"])
def toy(request):
    import torch
    from paper_1812_10659_amd import lola
    p = wl.PARAMS[request.param]
    print(f"[gpu-edges] params {p.name}", flush=True)
    ctx = lola.Context(p)
    octx = bfv.Context(p)
    steps = [1, 2, 4, -1, bfv.ROW_SWAP]
    gal = [bfv.galois_element(p.N, s) for s in steps]
    okeys = bfv.keygen(octx, SEED, gal)
    sk = ctx.keygen_secret(SEED)
    pk = ctx.keygen_public(SEED, sk)
    gks = {g: ctx.keygen_switch(SEED, sk, g) for g in gal}
    rlk = ctx.keygen_switch(SEED, sk, 0)
    rs = np.random.default_rng(7)
    msgs = [rs.integers(0, p.t, p.N).astype(np.uint64) for _ in range(4)]
    octs = [bfv.encrypt(octx, okeys, m, 21, k) for k, m in enumerate(msgs)]
    torch.cuda.synchronize()
    return dict(p=p, ctx=ctx, octx=octx, okeys=okeys, sk=sk, pk=pk, gks=gks, rlk=rlk, steps=steps, octs=octs)


def _up(ctx, limbs):
    from paper_1812_10659_amd import lola
    arr = np.stack([np.asarray(c, dtype=np.uint64) for c in limbs]).astype(np.uint32)
    return ctx.from_coeff(lola.from_numpy_u32(arr, ctx.device))


def _down(ctx, ct):
    from paper_1812_10659_amd import lola
    return lola.to_numpy_u32(ctx.to_coeff(ct)).astype(np.uint64)


def _code(excinfo):
    return excinfo.value.code


def test_empty_batches_are_no_ops(toy):
    from paper_1812_10659_amd import batched, lola
    ctx = toy["ctx"]
    assert ctx.keyswitch_batch([]) == []
    batched.mul_plain_batch(ctx, [], [], [])
    batched.mul_batch(ctx, [], [], [])
    batched.rotate_chains(ctx, [], [], [], [], {})
    import torch
    torch.cuda.synchronize()


@pytest.mark.parametrize("n_jobs", [1, 9, 13])
def test_ragged_keyswitch_batches(toy, n_jobs):
    """Batches of every size match the oracle job by job (the batched
    launches pad the job count to a multiple of the XCD count)."""
    ctx, octx, ok = toy["ctx"], toy["octx"], toy["okeys"]
    items, refs = [], []
    for k in range(n_jobs):
        step = toy["steps"][k % len(toy["steps"])]
        src = toy["octs"][k % len(toy["octs"])]
        g = bfv.galois_element(toy["p"].N, step)
        items.append((_up(ctx, src), toy["gks"][g], g))
        refs.append(np.stack(bfv.rotate(octx, src, step, ok)))
    outs = ctx.keyswitch_batch(items)
    for o, r in zip(outs, refs):
        assert np.array_equal(_down(ctx, o), r)


def test_persistent_chains_match_oracle(toy):
    """Uneven chains in one persistent launch, including a chain of one step."""
    from paper_1812_10659_amd import batched
    ctx, octx, ok = toy["ctx"], toy["octx"], toy["okeys"]
    chains = [[1, 2], [bfv.ROW_SWAP], [4, -1, 1]]
    ins = [_up(ctx, toy["octs"][k]) for k in range(len(chains))]
    outs = [ctx.empty_ct() for _ in chains]
    tmps = [ctx.empty_ct() for _ in chains]
    steps = [[bfv.galois_element(toy["p"].N, s) for s in ch] for ch in chains]
    batched.rotate_chains(ctx, ins, outs, tmps, steps, toy["gks"], n_wg=2)
    for k, ch in enumerate(chains):
        ref = toy["octs"][k]
        for s in ch:
            ref = bfv.rotate(octx, ref, s, ok)
        assert np.array_equal(_down(ctx, outs[k]), np.stack(ref))


def test_error_codes(toy):
    import torch
    from paper_1812_10659_amd import batched, lola
    ctx, p = toy["ctx"], toy["p"]
    ct = _up(ctx, toy["octs"][0])
    g1 = bfv.galois_element(p.N, 1)
    # an even Galois element is no automorphism of the ring
    with pytest.raises(lola.LolaError) as e:
        ctx.keyswitch_batch([(ct, toy["gks"][g1], 2)])
    assert _code(e) == -1
    # a ciphertext of size 4 cannot be decrypted
    with pytest.raises(lola.LolaError) as e:
        ctx.decrypt(toy["sk"], torch.zeros((4, p.L, p.N), dtype=torch.int32, device=ctx.device))
    assert _code(e) == -4
    # chains whose buffers alias
    with pytest.raises(lola.LolaError) as e:
        batched.rotate_chains(ctx, [ct], [ct], [ctx.empty_ct()], [[g1]], toy["gks"])
    assert _code(e) == -1
    # a transform of a prime the context does not have
    with pytest.raises(lola.LolaError) as e:
        ctx.ntt_limbs(torch.zeros((1, p.N), dtype=torch.int32, device=ctx.device), [99])
    assert _code(e) == -1
    # hoisted rotations: g = 1 or even, an output that is the input, a missing key
    for bad_g in (1, 2, 2 * p.N + 1):
        with pytest.raises(lola.LolaError) as e:
            ctx.rotate_hoisted(ct, [bad_g], [toy["gks"][g1]])
        assert _code(e) == -1
    garr = (ctypes.c_uint32 * 1)(g1)
    karr = (ctypes.c_void_p * 1)(toy["gks"][g1].data_ptr())
    oarr = (ctypes.c_void_p * 1)(ct.data_ptr())
    assert lola.lib().lola_rotate_hoisted(ctx.h, ct.data_ptr(), 1, garr, karr, oarr, lola._stream()) == -1
    karr0 = (ctypes.c_void_p * 1)(None)
    oarr2 = (ctypes.c_void_p * 1)(ctx.empty_ct().data_ptr())
    assert lola.lib().lola_rotate_hoisted(ctx.h, ct.data_ptr(), 1, garr, karr0, oarr2, lola._stream()) == -5
    assert lola.lib().lola_rotate_hoisted(ctx.h, ct.data_ptr(), 0, garr, karr, oarr2, lola._stream()) == 0
    # NTT variants: an index past the list, autotune sizes out of range
    nv = len(ctx.ntt_variants())
    with pytest.raises(lola.LolaError) as e:
        ctx.ntt_set_variant(nv)
    assert _code(e) == -1
    assert ctx.ntt_variant() == 0
    for n_limbs, reps in [(0, 1), (65537, 1), (4, 0), (4, 1001)]:
        with pytest.raises(lola.LolaError) as e:
            ctx.ntt_autotune(n_limbs=n_limbs, reps=reps)
        assert _code(e) == -1
    assert ctx.ntt_variant() == 0
    # a key switch without a key
    arr = (lola.KsDesc * 1)()
    out = ctx.empty_ct()
    arr[0] = lola.KsDesc(ct.data_ptr(), None, out.data_ptr(), g1, 0)
    assert lola.lib().lola_keyswitch_batch(ctx.h, arr, 1, lola._stream()) == -5
    torch.cuda.synchronize()


def test_plan_errors():
    import torch
    from paper_1812_10659_amd import lola, networks
    p = wl.PARAMS["n4096_3q"]
    x, W = wl.dense64_inputs()
    plan = lola.Plan(p, networks.dense64_layers(W))
    # constants loaded for another ring
    other = lola.Context(wl.PARAMS["toy1024"])
    with pytest.raises(lola.LolaError) as e:
        plan.load(other)
    assert e.value.code == -4
    # and for the same ring and primes with another key-switching shape (two
    # special primes): its keys and scratch differ
    other_k2 = lola.Context(wl.PARAMS["mnist_n16384_k2"])
    plan_k1 = lola.Plan(wl.PARAMS["mnist_n16384"], networks.mnist_small_layers(wl.mnist_small_weights()))
    with pytest.raises(lola.LolaError) as e:
        plan_k1.load(other_k2)
    assert e.value.code == -4
    other_k2.close()
    ctx = lola.Context(p)
    plan.load(ctx)
    sk = ctx.keygen_secret(3)
    pk = ctx.keygen_public(3, sk)
    gal = plan.galois()
    gks = [ctx.keygen_switch(3, sk, g) for g in gal]
    ins = [ctx.encrypt(pk, ctx.encode(np.zeros(p.N, dtype=np.int64)), 1, i) for i in range(plan.info["n_inputs"])]
    outs = [ctx.empty_ct() for _ in range(plan.info["n_outputs"])]
    # the plan squares, so a request without a relinearisation key is refused
    with pytest.raises(lola.LolaError) as e:
        plan.evaluate(ctx, [dict(rlk=None, gks=gks, inputs=ins, outputs=outs)])
    assert e.value.code == -5
    # a missing Galois key is refused
    rlk = ctx.keygen_switch(3, sk, 0)
    n = len(gal)
    gk_arr = (ctypes.c_void_p * n)(*([t.data_ptr() for t in gks[:-1]] + [None]))
    in_arr = (ctypes.c_void_p * len(ins))(*[t.data_ptr() for t in ins])
    out_arr = (ctypes.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
    req = (lola.Request * 1)()
    req[0] = lola.Request(rlk.data_ptr(), ctypes.cast(gk_arr, ctypes.POINTER(ctypes.c_void_p)),
                          ctypes.cast(in_arr, ctypes.POINTER(ctypes.c_void_p)),
                          ctypes.cast(out_arr, ctypes.POINTER(ctypes.c_void_p)))
    assert lola.lib().lola_evaluate(ctx.h, plan.h, req, 1, lola._stream()) == -5
    # an output that aliases an input
    with pytest.raises(lola.LolaError) as e:
        plan.evaluate(ctx, [dict(rlk=rlk, gks=gks, inputs=ins, outputs=[ins[0]] + outs[1:])])
    assert e.value.code == -1
    # a load that fails keeps the loaded constants, and a reload replaces them
    # (the next evaluation binds the new buffers): the words stay the same
    def words():
        plan.evaluate(ctx, [dict(rlk=rlk, gks=gks, inputs=ins, outputs=outs)])
        torch.cuda.synchronize()
        return [lola.to_numpy_u32(o).copy() for o in outs]
    ref = words()
    with pytest.raises(lola.LolaError) as e:
        plan.load(other)
    assert e.value.code == -4
    assert all(np.array_equal(a, b) for a, b in zip(words(), ref))
    plan.load(ctx)
    assert all(np.array_equal(a, b) for a, b in zip(words(), ref))
    # graph replay needs a stream of its own
    with pytest.raises(lola.LolaError) as e:
        plan.evaluate(ctx, [dict(rlk=rlk, gks=gks, inputs=ins, outputs=outs)], graph=True,
                      stream=torch.cuda.default_stream())
    assert e.value.code == -1
    # lanes: only 1 or 2
    for bad in (0, 3):
        with pytest.raises(lola.LolaError) as e:
            plan.set_lanes(bad)
        assert e.value.code == -1
    # an empty batch of requests is a no-op
    plan.evaluate(ctx, [])
    torch.cuda.synchronize()


def test_seeded_generation_is_deterministic(toy):
    """Keys and ciphertexts depend only on (seed, nonce), not on the context
    instance or on what ran before."""
    import torch
    from paper_1812_10659_amd import lola
    ctx2 = lola.Context(toy["p"])
    sk2 = ctx2.keygen_secret(SEED)
    pk2 = ctx2.keygen_public(SEED, sk2)
    ctx = toy["ctx"]
    assert torch.equal(ctx.export_sk(toy["sk"]), ctx2.export_sk(sk2))
    assert torch.equal(ctx.export_pk(toy["pk"]), ctx2.export_pk(pk2))
    m = ctx.encode(np.arange(toy["p"].N, dtype=np.int64) % toy["p"].t)
    a = ctx.encrypt(toy["pk"], m, 99, 5)
    b = ctx2.encrypt(pk2, ctx2.encode(np.arange(toy["p"].N, dtype=np.int64) % toy["p"].t), 99, 5)
    assert torch.equal(ctx.to_coeff(a), ctx2.to_coeff(b))
    c = ctx.encrypt(toy["pk"], m, 99, 6)
    assert not torch.equal(a, c)


def test_in_place_elementwise(toy):
    """Element-wise operations may write over an input."""
    ctx, octx = toy["ctx"], toy["octx"]
    a = _up(ctx, toy["octs"][0])
    b = _up(ctx, toy["octs"][1])
    ctx.add(a, b, out=a)
    ref = bfv.add(octx, toy["octs"][0], toy["octs"][1])
    assert np.array_equal(_down(ctx, a), np.stack(ref))
    ctx.mul_scalar(a, -3, out=a)
    ref = bfv.mul_scalar(octx, ref, -3)
    assert np.array_equal(_down(ctx, a), np.stack(ref))
