"""Pins of the oracle's CRT reconstruction and of the choice of plaintext
moduli for exact integer outputs of the MNIST-shaped network."""
import math
import random

import numpy as np
import pytest

from oracle import bfv, crt
from oracle import network as nw
from paper_1812_10659_amd import workloads as wl


def _is_prime(n):
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_brute_force_small_moduli():
    """Every integer of the centred range comes back from its residues."""
    for mods in ((3, 5, 7), (4, 9, 5), (2, 3), (11,)):
        M = math.prod(mods)
        for x in range(-(M // 2), (M + 1) // 2):
            assert crt.crt_combine([x % t for t in mods], mods) == x


def test_random_large_values_and_edges():
    mods = wl.MNIST_CRT_T
    M = math.prod(mods)
    rng = random.Random(5)
    xs = [rng.randrange(-(M // 2), (M + 1) // 2) for _ in range(300)]
    xs += [-(M // 2), (M - 1) // 2, 0, 1, -1]
    for x in xs:
        assert crt.crt_combine([x % t for t in mods], mods) == x
    # residues given as any representatives (negative or above t) are accepted
    x = 123456789123456789
    assert crt.crt_combine([x % t - t for t in mods], mods) == x


def test_rejects_non_coprime():
    with pytest.raises(ValueError):
        crt.crt_combine([1, 2], [6, 9])


def test_moduli_cover_the_network():
    """Primes = 1 mod 2N, pairwise distinct, and their product exceeds twice
    the largest |logit| the seeded weights allow, which in turn bounds the
    logits of actual images."""
    N = wl.PARAMS["mnist_n16384"].N
    for t in wl.MNIST_CRT_T:
        assert _is_prime(t) and t % (2 * N) == 1 and t < 2 ** 26
    assert len(set(wl.MNIST_CRT_T)) == len(wl.MNIST_CRT_T)
    w = wl.mnist_weights()
    bound = crt.mnist_logit_bound(w)
    assert math.prod(wl.MNIST_CRT_T) > 2 * bound
    for i in range(3):
        logits = nw.mnist_plain(wl.mnist_image(index=i), w)
        assert max(abs(int(v)) for v in logits) <= bound
    # the bound is attained in form: an all-255 image with sign-matched weights
    # would reach it, so it is not loose by more than the weights' spread
    assert bound < 2 ** 127


@pytest.mark.slow
@pytest.mark.parametrize("recipe", ["full", "shared"])
def test_tightest_modulus_keeps_a_noise_budget(recipe):
    """The modulus with the least room (t = 1179649) still decrypts the whole
    network exactly, with a positive noise budget, at seven data primes."""
    p = [q for q in wl.crt_params() if q.t == 1179649][0]
    ctx = bfv.Context(p)
    w = wl.mnist_weights()
    sched = nw.mnist_schedule(w, recipe=recipe)
    keys = bfv.keygen(ctx, 5, nw.galois_elements(sched))
    img = wl.mnist_image(index=0)
    cts = [bfv.encrypt(ctx, keys, bfv.encode(ctx, nw.dense_slots(m, p.N, p.t)), 1, i)
           for i, m in enumerate(nw.mnist_inputs(img))]
    outs, _ = nw.run_ciphertexts(ctx, keys, sched, cts)
    assert min(bfv.noise_budget(ctx, keys, o) for o in outs) > 1.0
    dec = [bfv.decode(ctx, bfv.decrypt(ctx, keys, o)) for o in outs]
    got = [int(dec[k][s]) for k, sl in enumerate(sched.out_slots) for s in sl]
    assert got == [int(v) for v in nw._mod(nw.mnist_plain(img, w), p.t)]
