"""Batched primitives at N=16384, L=8 on uniform residues: NTT round trips,
batched plaintext products, exact products with relinearisation, and uneven
rotation chains in one persistent launch -- each checked word for word
against the oracle on the same inputs; the wave-by-wave batched chains must
equal the persistent ones.  The small run keeps one prime per key-switching
digit; the full-size run is the bench's, with digits of two primes."""
import numpy as np
import pytest

from oracle import bfv
from paper_1812_10659_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_batched_primitives_match_oracle():
    import torch
    from paper_1812_10659_amd import batched, lola
    print("[gpu-batched] 24 ciphertexts, chains of <= 4 rotations, L=8", flush=True)
    r = batched.run_batched(n_ct=24, max_steps=4, tune=False, params="batch_n16384")
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


def _bitrev_perm(N):
    bits = N.bit_length() - 1
    return np.array([int(format(k, f"0{bits}b")[::-1], 2) for k in range(N)])


@pytest.fixture(scope="module")
def full_size():
    """The bench's configuration, run once: 512 ciphertexts, chains of 1..64
    rotations in one persistent launch, 256 products with relinearisation
    (key-switching digits of two primes); the oracle's keys for every step
    of the workload."""
    from paper_1812_10659_amd import batched
    print("[gpu-batched] 512 ciphertexts, full chains", flush=True)
    r = batched.run_batched(n_ct=512, tune=False)
    T = r.pop("_tensors")
    p = wl.PARAMS["batch_n16384_k2"]
    assert T["ctx"].K == 2
    octx = bfv.Context(p)
    need = sorted({bfv.galois_element(p.N, bfv.ROW_SWAP if s == 0 else int(s)) for row in T["steps"] for s in row})
    okeys = bfv.keygen(octx, T["seed"], need)
    steps = T["steps"]
    # eight seeded chains, the first of the longest always among them
    longest = max(range(len(steps)), key=lambda k: (len(steps[k]), -k))
    rest = [k for k in range(len(steps)) if k != longest]
    picks = [longest] + sorted(int(k) for k in wl.rng(T["seed"], 21).choice(rest, size=7, replace=False))
    return dict(r=r, T=T, p=p, octx=octx, okeys=okeys, picks=picks)


def test_full_size_batch_shape(full_size):
    r, T = full_size["r"], full_size["T"]
    assert r["ntt"]["roundtrip_exact"] and r["rotations_wavewise"]["equal_to_persistent"]
    assert r["rotations"] == sum(len(s) for s in T["steps"]) and max(len(s) for s in T["steps"]) == 64
    assert len(T["steps"][full_size["picks"][0]]) == 64


@pytest.mark.parametrize("slot", range(8))
def test_full_size_ciphertext_matches_oracle(full_size, slot):
    """One of eight seeded ciphertexts of the full-size run (slot 0: a
    64-rotation chain), every operation on it against the oracle word for
    word: the forward NTT of its limbs, its plaintext product, the product
    and relinearisation of its pair, and its whole rotation chain from the
    persistent launch."""
    from paper_1812_10659_amd import lola
    T, p, octx, okeys = full_size["T"], full_size["p"], full_size["octx"], full_size["okeys"]
    ctx, N, L = T["ctx"], p.N, p.L
    k = full_size["picks"][slot]
    print(f"[gpu-batched] ciphertext {k}: {len(T['steps'][k])} rotations", flush=True)
    down = lambda t: lola.to_numpy_u32(ctx.to_coeff(t)).astype(np.uint64)  # noqa: E731
    # forward transform of its 2L limbs: evaluation at the odd powers of the
    # minimal root of each prime, in bit-reversed order
    br = _bitrev_perm(N)
    raw = lola.to_numpy_u32(T["cts"][k]).reshape(2 * L, N)
    fwd = lola.to_numpy_u32(T["ntt_fwd"][2 * L * k:2 * L * (k + 1)])
    for row in range(2 * L):
        m = p.q[row % L]
        ev = np.empty(N, np.uint64)
        bfv.lib().or_eval_odd(raw[row].astype(np.uint64), ev, N, m, bfv.min_root_2n(m, N))
        assert np.array_equal(fwd[row].astype(np.uint64), ev[br]), f"NTT of limb {row}"
    x = list(down(T["cts"][k]))
    assert np.array_equal(down(T["prod"][k]), np.stack(bfv.mul_plain(octx, x, bfv.encode(octx, T["slots"][k]))))
    q = k // 2
    d = bfv.mul(octx, list(down(T["cts"][2 * q])), list(down(T["cts"][2 * q + 1])))
    assert np.array_equal(down(T["t3"][q]), np.stack(d)), "product of the pair"
    assert np.array_equal(down(T["rl"][q]), np.stack(bfv.relin(octx, d, okeys.rlk))), "relinearisation"
    for s in T["steps"][k]:
        x = bfv.rotate(octx, x, bfv.ROW_SWAP if s == 0 else int(s), okeys)
    assert np.array_equal(down(T["outs"][k]), np.stack(x)), f"chain {k}"
