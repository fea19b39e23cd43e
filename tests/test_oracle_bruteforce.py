"""Pins the oracle word for word against an independent pure-Python BFV
(tests/bruteforce_bfv.py) at tiny N, for every operation of the scheme."""
import numpy as np
import pytest

from oracle import bfv
from tests import bruteforce_bfv as bf


class _P:
    def __init__(self, N, t, q, P, P2=0):
        self.N, self.t, self.q, self.P, self.P2 = N, t, tuple(q), P, P2

    def special(self):
        return (self.P, self.P2) if self.P2 else self.P


# One digit per prime with one special prime; digits of two primes with two
# special primes (an odd and an even prime count: a one-prime last digit, and
# none).
TINY = [_P(16, 97, (193, 257, 353), 449), _P(32, 193, (257, 449, 577), 641),
        _P(16, 97, (193, 257, 353), 449, 577), _P(32, 193, (257, 449, 577, 641), 769, 1153)]


def _np(limbs):
    return np.array(limbs, dtype=np.uint64)


def _eq(ct_oracle, ct_bf):
    assert len(ct_oracle) == len(ct_bf)
    for a, b in zip(ct_oracle, ct_bf):
        assert np.array_equal(np.asarray(a, np.uint64), _np(b))


@pytest.fixture(params=TINY, ids=lambda p: f"N{p.N}_L{len(p.q)}" + ("_K2" if p.P2 else ""))
def setup(request):
    p = request.param
    ctx = bfv.Context(p)
    tiny = bf.Tiny(p.N, p.t, p.q, p.special())
    gs = [bfv.galois_element(p.N, 1), bfv.galois_element(p.N, -3), bfv.galois_element(p.N, bfv.ROW_SWAP)]
    seed = 0x1234_5678_9ABC
    keys = bfv.keygen(ctx, seed, gs)
    bkeys = tiny.keygen(seed, gs)
    rs = np.random.default_rng(p.N)
    m1 = rs.integers(0, p.t, p.N)
    m2 = rs.integers(0, p.t, p.N)
    ct1 = bfv.encrypt(ctx, keys, m1, 77, 3)
    ct2 = bfv.encrypt(ctx, keys, m2, 77, 4)
    bct1 = tiny.encrypt(bkeys, [int(v) for v in m1], 77, 3)
    bct2 = tiny.encrypt(bkeys, [int(v) for v in m2], 77, 4)
    return p, ctx, tiny, gs, keys, bkeys, (m1, m2), (ct1, ct2), (bct1, bct2)


def test_chacha_words_match(setup):
    assert list(bfv.stream_words(99, 5, 7, 2, 20)) == bf.words(99, 5, 7, 2, 20)


def test_keys_match(setup):
    p, ctx, tiny, gs, keys, bkeys, *_ = setup
    assert list(keys.sk.s) == bkeys["s"]
    assert np.array_equal(keys.pk0, _np(bkeys["pk0"]))
    assert np.array_equal(keys.pk1, _np(bkeys["pk1"]))
    b, a = bkeys["rlk"]
    nd, M = len(ctx.digits), len(ctx.moduli)
    assert keys.rlk.b.shape[:2] == (nd, M) and nd == (ctx.L + ctx.K - 1) // ctx.K
    for i in range(nd):
        for j in range(M):
            assert list(keys.rlk.b[i, j]) == b[i][j]
            assert list(keys.rlk.a[i, j]) == a[i][j]
    for g in gs:
        b, a = bkeys["gal"][g]
        assert all(list(keys.galois[g].b[i, j]) == b[i][j]
                   for i in range(nd) for j in range(M))


def test_encode_decode_match(setup):
    p, ctx, tiny, *_ , (m1, m2), _c, _b = setup
    assert list(bfv.decode(ctx, m1)) == tiny.decode([int(v) for v in m1])
    v = [int(x) for x in np.random.default_rng(5).integers(0, p.t, p.N)]
    assert list(bfv.encode(ctx, v)) == tiny.encode(v)


def test_encrypt_decrypt_match(setup):
    p, ctx, tiny, gs, keys, bkeys, (m1, m2), (c1, c2), (b1, b2) = setup
    _eq(c1, b1)
    _eq(c2, b2)
    assert list(bfv.decrypt(ctx, keys, c1)) == tiny.decrypt(bkeys, b1)


def test_linear_ops_match(setup):
    p, ctx, tiny, gs, keys, bkeys, (m1, m2), (c1, c2), (b1, b2) = setup
    _eq(bfv.add(ctx, c1, c2), tiny.add(b1, b2))
    _eq(bfv.add_plain(ctx, c1, m2), tiny.add_plain(b1, [int(v) for v in m2]))
    _eq(bfv.mul_plain(ctx, c1, m2), tiny.mul_plain(b1, [int(v) for v in m2]))
    for w in (0, 1, -1, 5, p.t - 2, p.t // 2 + 1):
        _eq(bfv.mul_scalar(ctx, c1, w), tiny.mul_scalar(b1, w))


def test_mul_relin_match(setup):
    p, ctx, tiny, gs, keys, bkeys, (m1, m2), (c1, c2), (b1, b2) = setup
    d = bfv.mul(ctx, c1, c2)
    bd = tiny.mul(b1, b2)
    _eq(d, bd)
    _eq(bfv.relin(ctx, d, keys.rlk), tiny.relin(bd, bkeys))
    _eq(bfv.mul(ctx, c1, c1), tiny.mul(b1, b1))


def test_rotate_match(setup):
    p, ctx, tiny, gs, keys, bkeys, (m1, m2), (c1, c2), (b1, b2) = setup
    for step in (1, -3, bfv.ROW_SWAP):
        g = bfv.galois_element(p.N, step)
        _eq(bfv.rotate(ctx, c1, step, keys), tiny.rotate(b1, g, bkeys))


def test_rotate_hoisted_match(setup):
    """The hoisted rotation (digits taken before the automorphism) word for
    word, and it decrypts like the plain rotation while its words differ."""
    p, ctx, tiny, gs, keys, bkeys, (m1, m2), (c1, c2), (b1, b2) = setup
    for step in (1, -3, bfv.ROW_SWAP):
        g = bfv.galois_element(p.N, step)
        h = bfv.rotate_hoisted(ctx, c1, step, keys)
        _eq(h, tiny.rotate_hoisted(b1, g, bkeys))
        r = bfv.rotate(ctx, c1, step, keys)
        assert list(bfv.decrypt(ctx, keys, h)) == list(bfv.decrypt(ctx, keys, r))
        assert any(not np.array_equal(x, y) for x, y in zip(h, r))


def test_decrypt_of_size3_match(setup):
    p, ctx, tiny, gs, keys, bkeys, (m1, m2), (c1, c2), (b1, b2) = setup
    d = bfv.mul(ctx, c1, c2)
    assert list(bfv.decrypt(ctx, keys, d)) == tiny.decrypt(bkeys, tiny.mul(b1, b2))


def test_256_bit_seed_keys_and_encryption_match():
    """A seed with all eight key words set (a full 256-bit ChaCha20 key): the
    oracle's keys and encryption equal the brute force's word for word, and
    differ from those of the same seed's low 64 bits alone."""
    p = TINY[0]
    ctx = bfv.Context(p)
    tiny = bf.Tiny(p.N, p.t, p.q, p.special())
    g = [bfv.galois_element(p.N, 1)]
    seed = int.from_bytes(bytes(range(1, 33)), "little")
    keys, bkeys = bfv.keygen(ctx, seed, g), tiny.keygen(seed, g)
    assert list(keys.sk.s) == bkeys["s"]
    assert np.array_equal(keys.pk0, _np(bkeys["pk0"])) and np.array_equal(keys.pk1, _np(bkeys["pk1"]))
    b, a = bkeys["gal"][g[0]]
    for i in range(len(ctx.digits)):
        for j in range(len(ctx.moduli)):
            assert list(keys.galois[g[0]].b[i, j]) == b[i][j] and list(keys.galois[g[0]].a[i, j]) == a[i][j]
    m = np.arange(p.N) % p.t
    _eq(bfv.encrypt(ctx, keys, m, seed + 5, 2), tiny.encrypt(bkeys, [int(v) for v in m], seed + 5, 2))
    low = bfv.keygen(ctx, seed & ((1 << 64) - 1), g)
    assert not np.array_equal(low.pk0, keys.pk0)
    assert list(bfv.seed_key(seed)) == [int.from_bytes(bytes(range(4 * k + 1, 4 * k + 5)), "little") for k in range(8)]
