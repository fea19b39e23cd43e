"""Batched primitives at N=16384, L=8 on uniform residues: NTT round trips,
batched plaintext products, exact products with relinearisation, and uneven
rotation chains in one persistent launch -- each checked word for word
against the oracle on the same inputs; the wave-by-wave batched chains must
equal the persistent ones."""
import numpy as np
import pytest

from oracle import bfv
from paper_1812_10659_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_batched_primitives_match_oracle():
    import torch
    from paper_1812_10659_amd import batched, lola
    print("[gpu-batched] 24 ciphertexts, chains of <= 4 rotations, L=8", flush=True)
    r = batched.run_batched(n_ct=24, max_steps=4, tune=False)
    T = r.pop("_tensors")
    ctx = T["ctx"]
    assert r["ntt"]["roundtrip_exact"]
    assert r["rotations_wavewise"]["equal_to_persistent"]
    p = wl.PARAMS["batch_n16384"]
    octx = bfv.Context(p)
    steps = T["steps"]
    need = sorted({bfv.galois_element(p.N, bfv.ROW_SWAP if s == 0 else int(s)) for row in steps[:4] for s in row})
    okeys = bfv.keygen(octx, T["seed"], need)
    down = lambda t: lola.to_numpy_u32(ctx.to_coeff(t)).astype(np.uint64)  # noqa: E731
    oc = [list(down(T["cts"][k])) for k in range(4)]
    for k in range(4):
        m = bfv.encode(octx, T["slots"][k])
        assert np.array_equal(down(T["prod"][k]), np.stack(bfv.mul_plain(octx, oc[k], m)))
        x = oc[k]
        for s in steps[k]:
            x = bfv.rotate(octx, x, bfv.ROW_SWAP if s == 0 else int(s), okeys)
        assert np.array_equal(down(T["outs"][k]), np.stack(x)), f"chain {k}"
    for k in range(2):
        d = bfv.mul(octx, oc[2 * k], oc[2 * k + 1])
        assert np.array_equal(down(T["t3"][k]), np.stack(d))
        assert np.array_equal(down(T["rl"][k]), np.stack(bfv.relin(octx, d, okeys.rlk)))


def test_batched_primitives_full_size_sampled():
    """The bench's configuration (512 ciphertexts, chains of 1..64 rotations
    in one persistent launch, 256 products with relinearisation): sampled
    outputs against the oracle -- the two shortest chains, the first and last
    plaintext products and one product pair -- and the wave-by-wave chains
    equal to the persistent ones everywhere."""
    from paper_1812_10659_amd import batched, lola
    print("[gpu-batched] 512 ciphertexts, full chains, sampled", flush=True)
    r = batched.run_batched(n_ct=512, tune=False)
    T = r.pop("_tensors")
    ctx = T["ctx"]
    assert r["ntt"]["roundtrip_exact"] and r["rotations_wavewise"]["equal_to_persistent"]
    assert r["rotations"] == sum(len(s) for s in T["steps"]) and max(len(s) for s in T["steps"]) == 64
    p = wl.PARAMS["batch_n16384"]
    octx = bfv.Context(p)
    steps = T["steps"]
    chains = sorted(range(len(steps)), key=lambda k: (len(steps[k]), k))[:2]
    need = sorted({bfv.galois_element(p.N, bfv.ROW_SWAP if s == 0 else int(s)) for k in chains for s in steps[k]})
    okeys = bfv.keygen(octx, T["seed"], need)
    down = lambda t: lola.to_numpy_u32(ctx.to_coeff(t)).astype(np.uint64)  # noqa: E731
    n = len(T["cts"])
    for k in sorted(set(chains + [0, n - 1])):
        x = list(down(T["cts"][k]))
        if k in (0, n - 1):
            m = bfv.encode(octx, T["slots"][k])
            assert np.array_equal(down(T["prod"][k]), np.stack(bfv.mul_plain(octx, x, m))), f"product {k}"
        if k in chains:
            for s in steps[k]:
                x = bfv.rotate(octx, x, bfv.ROW_SWAP if s == 0 else int(s), okeys)
            assert np.array_equal(down(T["outs"][k]), np.stack(x)), f"chain {k} ({len(steps[k])} steps)"
    q = n // 2 - 1
    d = bfv.mul(octx, list(down(T["cts"][2 * q])), list(down(T["cts"][2 * q + 1])))
    assert np.array_equal(down(T["t3"][q]), np.stack(d))
    assert np.array_equal(down(T["rl"][q]), np.stack(bfv.relin(octx, d, okeys.rlk)))
