"""Pins of the oracle's scheme: slot encoding, rotations, homomorphic
properties, the key-switching error bound, noise budgets, parameter security,
and the paper's worked examples and tables."""
import math
import os

import numpy as np
import pytest

from oracle import bfv
from oracle import network as nw
from paper_1812_10659_amd import workloads as wl
from tests import bruteforce_bfv as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


@pytest.fixture(scope="module")
def ctx1024():
    return bfv.Context(wl.PARAMS["toy1024"])


@pytest.fixture(scope="module")
def keys1024(ctx1024):
    steps = [1, 2, 4, 8, 16, 32, 64, 128, 256, -1, -5, bfv.ROW_SWAP]
    return bfv.keygen(ctx1024, 2024, [bfv.galois_element(1024, s) for s in steps])


# ------------------------------------------------------------- P2 slots ----
def test_slot_exponents_are_odd_residue_permutation():
    for N in (16, 1024, 16384):
        ctx_e = {(pow(2 * N - 1, r, 2 * N) * pow(3, i, 2 * N)) % (2 * N)
                 for r in range(2) for i in range(N // 2)}
        assert ctx_e == set(range(1, 2 * N, 2))


@pytest.mark.parametrize("name", ["toy1024", "n4096_3q", "mnist_n16384"])
def test_encode_decode_roundtrip_and_homomorphism(name):
    ctx = bfv.Context(wl.PARAMS[name])
    rs = np.random.default_rng(1)
    v = rs.integers(0, ctx.t, ctx.N)
    w = rs.integers(0, ctx.t, ctx.N)
    mv, mw = bfv.encode(ctx, v), bfv.encode(ctx, w)
    assert np.array_equal(bfv.decode(ctx, mv), v)
    assert mv.max() < ctx.t
    # encode is a ring homomorphism: encode(v) * encode(w) = encode(v . w) in R_t
    assert np.array_equal(bfv.poly_mul(mv, mw, ctx.t), bfv.encode(ctx, (v * w) % ctx.t))
    # a constant polynomial sets every slot to the constant (Sec. 4.2.1 footnote)
    c = np.zeros(ctx.N, np.uint64); c[0] = 12345 % ctx.t
    assert np.all(bfv.decode(ctx, c) == 12345 % ctx.t)


def test_zeta_is_smallest_primitive_root():
    for p in wl.PARAMS.values():
        z = bfv.min_root_2n(p.t, p.N)
        assert pow(z, p.N, p.t) == p.t - 1
        assert all(pow(g, p.N, p.t) != p.t - 1 for g in range(2, min(z, 5000)))


# ---------------------------------------------------------- P3 rotations ----
@pytest.mark.parametrize("name", ["toy1024", "mnist_n16384"])
def test_automorphism_rotates_slots(name):
    ctx = bfv.Context(wl.PARAMS[name])
    N = ctx.N
    v = np.random.default_rng(2).integers(0, ctx.t, N)
    m = bfv.encode(ctx, v)
    k = 1
    while k < N // 2:
        g = bfv.galois_element(N, k)
        got = bfv.decode(ctx, bfv.automorph(m, ctx.t, g))
        assert np.array_equal(got, nw.rotate_slots(v, k))
        assert np.array_equal(nw.rotate_slots(v, k)[:N // 2], np.roll(v[:N // 2], -k))
        k *= 2 if name == "toy1024" else 64
    got = bfv.decode(ctx, bfv.automorph(m, ctx.t, 2 * N - 1))
    assert np.array_equal(got, np.concatenate([v[N // 2:], v[:N // 2]]))


# -------------------------------------------------------- P4 homomorphism ----
def test_homomorphic_ops_and_budgets(ctx1024, keys1024):
    ctx, keys = ctx1024, keys1024
    rs = np.random.default_rng(3)
    v, w = rs.integers(0, ctx.t, ctx.N), rs.integers(0, ctx.t, ctx.N)
    c1 = bfv.encrypt(ctx, keys, bfv.encode(ctx, v), 5, 1)
    c2 = bfv.encrypt(ctx, keys, bfv.encode(ctx, w), 5, 2)
    dec = lambda c: bfv.decode(ctx, bfv.decrypt(ctx, keys, c))  # noqa: E731
    b0 = bfv.noise_budget(ctx, keys, c1)
    assert b0 > 30
    assert np.array_equal(dec(c1), v)
    assert np.array_equal(dec(bfv.add(ctx, c1, c2)), (v + w) % ctx.t)
    assert np.array_equal(dec(bfv.add_plain(ctx, c1, bfv.encode(ctx, w))), (v + w) % ctx.t)
    mp = bfv.mul_plain(ctx, c1, bfv.encode(ctx, w))
    assert np.array_equal(dec(mp), (v * w) % ctx.t)
    assert np.array_equal(dec(bfv.mul_scalar(ctx, c1, -7)), (v * -7) % ctx.t)
    d3 = bfv.mul(ctx, c1, c2)
    assert np.array_equal(dec(d3), (v * w) % ctx.t)
    r = bfv.relin(ctx, d3, keys.rlk)
    assert np.array_equal(dec(r), (v * w) % ctx.t)
    for step in (1, 256, -5, bfv.ROW_SWAP):
        assert np.array_equal(dec(bfv.rotate(ctx, c1, step, keys)), nw.rotate_slots(v, step))
    # budgets never grow along a chain of operations
    chain = [c1]
    chain.append(bfv.mul_plain(ctx, chain[-1], bfv.encode(ctx, w)))
    chain.append(bfv.rotate(ctx, chain[-1], 1, keys))
    chain.append(bfv.square(ctx, chain[-1], keys))
    bud = [bfv.noise_budget(ctx, keys, c) for c in chain]
    assert all(b2 <= b1 + 1e-9 for b1, b2 in zip(bud, bud[1:])), bud
    assert bud[-1] > 0


# ---------------------------------------------------- P5 key-switch bound ----
def test_keyswitch_error_bound(ctx1024, keys1024):
    """k0 + k1 s - x s' is small: |.| <= (L N q_max B_e + P N)/P + N."""
    ctx, keys = ctx1024, keys1024
    rs = np.random.default_rng(9)
    x = np.stack([rs.integers(0, q, ctx.N, dtype=np.uint64) for q in ctx.q])
    g = bfv.galois_element(ctx.N, 1)
    ksk = keys.galois[g]
    k0, k1 = bfv.keyswitch(ctx, x, ksk)
    s_l = ctx.small_to_limbs(keys.sk.s)
    sg = np.stack([bfv.automorph(s_l[j], q, g) for j, q in enumerate(ctx.q)])
    diff = []
    for j, q in enumerate(ctx.q):
        k1s = bfv.poly_mul(k1[j], s_l[j], q)
        xs = bfv.poly_mul(x[j], sg[j], q)
        diff.append((k0[j] + k1s + (q - xs)) % q)
    err = ctx.centred_lift(diff)
    bound = (ctx.L * ctx.N * max(ctx.q) * 21 + ctx.P * ctx.N) // ctx.P + ctx.N
    assert max(abs(int(e)) for e in err) <= bound
    assert max(abs(int(e)) for e in err) < ctx.Q // (2 * ctx.t)


def test_two_prime_digits_decrypt_and_meet_their_bound():
    """Key switching with digits of two primes and two special primes at
    N = 1024: rotations (plain and hoisted) and relinearisation decrypt to the
    slot results, the error of a key switch stays under
    (d N max Q_d B_e + P N)/P + N for d digits of modulus Q_d, and the noise
    budget left by a rotation is within a bit of the one-prime-digit set's
    (P grows with the digits)."""
    ctx = bfv.Context(wl.PARAMS["toy1024_k2"])
    assert ctx.K == 2 and ctx.digits == [[0, 1], [2]]
    steps = [1, -5, bfv.ROW_SWAP]
    keys = bfv.keygen(ctx, 2025, [bfv.galois_element(1024, s) for s in steps])
    rs = np.random.default_rng(4)
    v, w = rs.integers(0, ctx.t, ctx.N), rs.integers(0, ctx.t, ctx.N)
    c1 = bfv.encrypt(ctx, keys, bfv.encode(ctx, v), 6, 1)
    c2 = bfv.encrypt(ctx, keys, bfv.encode(ctx, w), 6, 2)
    dec = lambda c: bfv.decode(ctx, bfv.decrypt(ctx, keys, c))  # noqa: E731
    for step in steps:
        assert np.array_equal(dec(bfv.rotate(ctx, c1, step, keys)), nw.rotate_slots(v, step))
        assert np.array_equal(dec(bfv.rotate_hoisted(ctx, c1, step, keys)), nw.rotate_slots(v, step))
    assert np.array_equal(dec(bfv.relin(ctx, bfv.mul(ctx, c1, c2), keys.rlk)), (v * w) % ctx.t)
    x = np.stack([rs.integers(0, q, ctx.N, dtype=np.uint64) for q in ctx.q])
    g = bfv.galois_element(ctx.N, 1)
    k0, k1 = bfv.keyswitch(ctx, x, keys.galois[g])
    s_l = ctx.small_to_limbs(keys.sk.s)
    diff = []
    for j, q in enumerate(ctx.q):
        xs = bfv.poly_mul(x[j], bfv.automorph(s_l[j], q, g), q)
        diff.append((k0[j] + bfv.poly_mul(k1[j], s_l[j], q) + (q - xs)) % q)
    err = max(abs(int(e)) for e in ctx.centred_lift(diff))
    qd = max(math.prod(ctx.q[k] for k in dg) for dg in ctx.digits)
    assert err <= (len(ctx.digits) * ctx.N * qd * 21 + ctx.P * ctx.N) // ctx.P + ctx.N
    c1_ = bfv.Context(wl.PARAMS["toy1024"])
    k1_ = bfv.keygen(c1_, 2025, [g])
    r1 = bfv.rotate(c1_, bfv.encrypt(c1_, k1_, bfv.encode(c1_, v), 6, 1), 1, k1_)
    b2, b1 = bfv.noise_budget(ctx, keys, bfv.rotate(ctx, c1, 1, keys)), bfv.noise_budget(c1_, k1_, r1)
    assert abs(b2 - b1) < 1.0, (b2, b1)


# ---------------------------------------------- parameters and failure ----
def test_parameter_sets_meet_security_caps():
    for p in wl.PARAMS.values():
        bits = sum(math.log2(x) for x in (*p.q, *p.special))
        if not p.insecure_ok:
            assert bits <= wl.SECURITY_CAP_LOG2[p.N], p.name
        assert math.gcd(p.t, math.prod(p.q)) == 1
        assert len(set((*p.q, *p.special))) == p.L + len(p.special)
        assert all(bf_is_prime(x) for x in (*p.q, *p.special, p.t))


def bf_is_prime(n):
    return bfv._is_prime(n) and all(n % d for d in range(2, 1000) if d * d <= n and d < n)


def test_literal_two_prime_n4096_fails_noise_check():
    """With q ~ 2^60 the square activation exhausts the noise budget: the
    budget drops to ~0 and decryption no longer matches (the failure the
    working N=4096 set with three primes avoids)."""
    x, W = wl.dense64_inputs()
    out = {}
    for name in ("n4096_2q", "n4096_3q"):
        ctx = bfv.Context(wl.PARAMS[name])
        sc = nw.dense64_schedule(W)
        keys = bfv.keygen(ctx, wl.key_seed(0), nw.galois_elements(sc))
        inp = nw.dense_slots(nw.dense64_inputs(x, 4096)[0], 4096, ctx.t)
        cts = [bfv.encrypt(ctx, keys, bfv.encode(ctx, inp), wl.enc_seed(0), 0)]
        res, _ = nw.run_ciphertexts(ctx, keys, sc, cts)
        dec = bfv.decode(ctx, bfv.decrypt(ctx, keys, res[0]))
        exp = nw._mod(nw.dense64_plain(x, W), ctx.t)
        out[name] = (bfv.noise_budget(ctx, keys, res[0]), all(dec[64 * j] == exp[j] for j in range(64)))
    assert out["n4096_2q"][0] < 1.0 and not out["n4096_2q"][1]
    assert out["n4096_3q"][0] > 1.0 and out["n4096_3q"][1]


# ------------------------------------------------- P7 paper examples ----
class _N8:
    N, t, q, P = 8, 17, tuple(wl.PRIMES_16384[:3]), wl.PRIMES_16384[3]


def test_footnote_dot_product_on_ciphertexts():
    """N = 8: a slot row is the paper's 4-vector; its rotation of size k is
    rotate(-k) here (entry i moves to i+k)."""
    ctx = bfv.Context(_N8)
    keys = bfv.keygen(ctx, 11, [bfv.galois_element(8, -1), bfv.galois_element(8, -2),
                                bfv.galois_element(8, 1), bfv.galois_element(8, 2)])
    v = np.array([3, 1, 4, 1, 0, 0, 0, 0]); w = np.array([2, 7, 1, 8, 0, 0, 0, 0])
    p = (v * w) % ctx.t
    lines = {ln[0]: ln[1:] for ln in _golden_lines("paper_footnote_dot_product.txt")}

    def expected(spec):
        return [sum(int(p[int(k) - 1]) for k in e.split("+")) % ctx.t for e in spec]

    ct = bfv.mul_plain(ctx, bfv.encrypt(ctx, keys, bfv.encode(ctx, v), 1, 1), bfv.encode(ctx, w))
    dec = lambda c: list(bfv.decode(ctx, bfv.decrypt(ctx, keys, c))[:4])  # noqa: E731
    r1 = bfv.add(ctx, ct, bfv.rotate(ctx, ct, -1, keys))
    assert dec(r1) == expected(lines["after_rot1"])
    r2 = bfv.add(ctx, r1, bfv.rotate(ctx, r1, -2, keys))
    assert dec(r2) == expected(lines["after_rot2"])
    # the same sums with left rotations put each window sum at its first entry
    l1 = bfv.add(ctx, ct, bfv.rotate(ctx, ct, 1, keys))
    l2 = bfv.add(ctx, l1, bfv.rotate(ctx, l1, 2, keys))
    assert dec(l2) == expected(lines["after_rot2"])


def test_footnote_stacked_row_major():
    ctx = bfv.Context(_N8)
    keys = bfv.keygen(ctx, 12, [bfv.galois_element(8, -1), bfv.galois_element(8, 1)])
    w11, w12, w21, w22, v1, v2 = 2, 3, 5, 7, 4, 6
    env = dict(w11=w11, w12=w12, w21=w21, w22=w22, v1=v1, v2=v2)
    stacked = np.array([v1, v2, v1, v2, 0, 0, 0, 0]); flat = np.array([w11, w12, w21, w22, 0, 0, 0, 0])
    ct = bfv.mul_plain(ctx, bfv.encrypt(ctx, keys, bfv.encode(ctx, stacked), 1, 1), bfv.encode(ctx, flat))
    r = bfv.add(ctx, ct, bfv.rotate(ctx, ct, -1, keys))     # paper's direction
    d = bfv.decode(ctx, bfv.decrypt(ctx, keys, r))
    for _, entry, expr in _golden_lines("paper_footnote_stacked_2x2.txt"):
        assert d[int(entry) - 1] == eval(expr, {}, env) % ctx.t  # noqa: S307 (fixture arithmetic)
    # left-rotation convention: the same values one entry earlier
    rl = bfv.add(ctx, ct, bfv.rotate(ctx, ct, 1, keys))
    dl = bfv.decode(ctx, bfv.decrypt(ctx, keys, rl))
    for _, entry, expr in _golden_lines("paper_footnote_stacked_2x2.txt"):
        assert dl[int(entry) - 2] == eval(expr, {}, env) % ctx.t  # noqa: S307


def test_footnote_convolution_representation():
    A = np.arange(1, 17).reshape(4, 4) * 10 + 0  # value at (i,j) 1-based = 10*(4(i-1)+(j-1)+1)
    msgs = nw.conv_representation(A, 2, 2)
    for name, *cells in _golden_lines("paper_footnote_conv_repr.txt"):
        k = int(name[1:]) - 1
        exp = [A[int(c.split(",")[0]) - 1, int(c.split(",")[1]) - 1] for c in cells]
        assert list(msgs[k]) == exp
    # sum_j w_j M^j is the strided convolution
    wgt = np.array([[1, -2], [3, 5]])
    conv = sum(wgt[a, b] * msgs[2 * a + b] for a in range(2) for b in range(2))
    direct = [int((A[2 * y:2 * y + 2, 2 * x:2 * x + 2] * wgt).sum()) for y in range(2) for x in range(2)]
    assert list(conv) == direct


# --------------------------------------------------------- P8 tables ----
def test_mnist_schedule_matches_table_shapes():
    wts = wl.mnist_weights()
    img = wl.mnist_image()
    sc = nw.mnist_schedule(wts)
    tab = {ln[0]: ln[1] for ln in _golden_lines("paper_tables_mnist.txt")}
    n_in, dim = map(int, tab["conv_input"].split("x"))
    ins = nw.mnist_inputs(img)
    assert len(ins) == n_in == sc.n_inputs and all(len(m) == dim for m in ins)
    # conv: 25 scalar products per map, 5 maps
    assert sc.count("mul_scalar") == 25 * int(tab["conv_output"].split("x")[0])
    squares = [i for i, op in enumerate(sc.ops) if op[0] == "square"]
    assert len(squares) == 2
    rot_before_sq1 = sum(1 for op in sc.ops[:squares[0]] if op[0] == "rotate")
    assert rot_before_sq1 == int(tab["combine_maps_rotations"])
    _, reg = nw.run_slots(sc, ins, 1146881)
    sq1_in = sc.ops[squares[0]][2]
    n1, d1 = map(int, tab["square1_input"].split("x"))
    assert np.count_nonzero(reg[sq1_in]) <= d1 and np.count_nonzero(reg[sq1_in][d1:]) == 0
    assert int(tab["square1_multiplications"]) == 1
    # stacked: 16 copies of the 845 values
    stack_reg = sc.ops[squares[0] + 8][1]
    ns, ds = map(int, tab["stacked"].split("x"))
    assert ds == 16 * 845
    v = reg[stack_reg]
    assert all(np.array_equal(v[1024 * c:1024 * c + 845], v[:845]) for c in range(16))
    # 7 rounds of up to 16 outputs
    nr, dr = map(int, tab["dense1_rounds"].split("x"))
    assert sum(1 for op in sc.ops if op[0] == "mul_plain") == 2 * nr + 10
    n2_, d2_ = map(int, tab["square2_input"].split("x"))
    assert nr * dr >= d2_ > (nr - 1) * dr
    assert len(sc.outputs) == int(tab["output"].split("x")[0])


# ---------------------------------------------------- P9 end to end ----
def test_slot_schedules_equal_plain_networks():
    x, W = wl.dense64_inputs()
    outs, _ = nw.run_slots(nw.dense64_schedule(W), nw.dense64_inputs(x, 4096), 65537)
    exp = nw._mod(nw.dense64_plain(x, W), 65537)
    assert all(outs[0][64 * j] == exp[j] for j in range(64))
    wts, img = wl.mnist_weights(), wl.mnist_image()
    outs, _ = nw.run_slots(nw.mnist_schedule(wts), nw.mnist_inputs(img), 1146881)
    assert [int(o[0]) for o in outs] == list(nw._mod(nw.mnist_plain(img, wts), 1146881))
    outs, _ = nw.run_slots(nw.mnist_schedule(wts, recipe="shared"), nw.mnist_inputs(img), 1146881)
    assert [int(outs[0][8 * o]) for o in range(10)] == list(nw._mod(nw.mnist_plain(img, wts), 1146881))
    hw, f = wl.head_weights(), wl.head_features(4)
    outs, _ = nw.run_slots(nw.head_schedule(hw), nw.head_inputs(f), 1146881)
    for q in range(4):
        exp = nw._mod(nw.head_plain(f[q], hw), 1146881)
        assert [int(outs[o][4096 * q]) for o in range(10)] == list(exp)


@pytest.mark.parametrize("index", [0, 1, 4])
def test_shared_reduction_equals_full_at_valid_slots(index):
    """The two reduction recipes of the MNIST networks (full: every round summed
    over its block; shared: rounds summed within groups, combined, one shared
    tail) give the same hidden vector at every valid slot P c + rho of the
    second square's input, and the same logits; the shared schedule's garbage
    slots differ.  Also for LoLa-Dense (P = 2048, 13 rounds, groups of 16)."""
    wts, img = wl.mnist_weights(), wl.mnist_image(index=index)
    for mk, ins, P, C, R, t in [(nw.mnist_schedule, nw.mnist_inputs(img), 1024, 16, 7, 1146881),
                                (nw.mnist_dense_schedule, nw.mnist_dense_inputs(img), 2048, 8, 13, 1146881)]:
        hid = {}
        res = {}
        for rec in ("full", "shared"):
            sc = mk(wts, recipe=rec)
            outs, reg = nw.run_slots(sc, ins, t)
            hid[rec] = reg[[op for op in sc.ops if op[0] == "square"][1][2]]
            res[rec] = [int(outs[k][s]) for k, sl in enumerate(sc.out_slots) for s in sl]
        valid = [P * c + rho for rho in range(R) for c in range(C) if C * rho + c < 100]
        assert np.array_equal(hid["full"][valid], hid["shared"][valid])
        assert not np.array_equal(hid["full"], hid["shared"])
        assert res["full"] == res["shared"] == list(nw._mod(nw.mnist_plain(img, wts), t))


def test_dense64_ciphertext_schedule_end_to_end():
    ctx = bfv.Context(wl.PARAMS["n4096_3q"])
    x, W = wl.dense64_inputs()
    sc = nw.dense64_schedule(W)
    keys = bfv.keygen(ctx, wl.key_seed(0), nw.galois_elements(sc))
    inp = nw.dense_slots(nw.dense64_inputs(x, 4096)[0], 4096, ctx.t)
    res, reg = nw.run_ciphertexts(ctx, keys, sc, [bfv.encrypt(ctx, keys, bfv.encode(ctx, inp), 1, 0)], keep=True)
    slots, sreg = nw.run_slots(sc, nw.dense64_inputs(x, 4096), ctx.t)
    # every slot of every register equals the slot interpreter
    for r in reg:
        assert np.array_equal(bfv.decode(ctx, bfv.decrypt(ctx, keys, reg[r])), sreg[r])


@pytest.mark.slow
@pytest.mark.parametrize("recipe", ["full", "shared"])
def test_mnist_ciphertext_schedule_end_to_end(recipe):
    ctx = bfv.Context(wl.PARAMS["mnist_n16384"])
    wts, img = wl.mnist_weights(), wl.mnist_image()
    sc = nw.mnist_schedule(wts, recipe=recipe)
    keys = bfv.keygen(ctx, wl.key_seed(1), nw.galois_elements(sc))
    ins = nw.mnist_inputs(img)
    cts = [bfv.encrypt(ctx, keys, bfv.encode(ctx, nw.dense_slots(m, ctx.N, ctx.t)), wl.enc_seed(1), i)
           for i, m in enumerate(ins)]
    outs, _ = nw.run_ciphertexts(ctx, keys, sc, cts)
    slots, _ = nw.run_slots(sc, ins, ctx.t)
    for o, s in zip(outs, slots):
        assert np.array_equal(bfv.decode(ctx, bfv.decrypt(ctx, keys, o)), s)
        assert bfv.noise_budget(ctx, keys, o) > 1.0
    got = [int(slots[k][s]) for k, sl in enumerate(sc.out_slots) for s in sl]
    assert got == list(nw._mod(nw.mnist_plain(img, wts), ctx.t))


def test_bruteforce_chacha_quarter_round_vector():
    rows = {ln[0]: ln[1:] for ln in _golden_lines("chacha20_rfc8439.txt")}
    assert [f"{x:08x}" for x in bf.quarter_round(*[int(w, 16) for w in rows["qr_in"]])] == rows["qr_out"]
    key = [int(w, 16) for w in rows["key"]]
    out = bf.chacha20_block(key, 1, [int(w, 16) for w in rows["nonce"]])
    assert [f"{x:08x}" for x in out] == rows["out"]


@pytest.mark.parametrize("sparse", [False, True])
def test_dense_chain_ciphertexts_decrypt_to_network(sparse):
    """Sparse vector - column major and dense vector - row major (Sec. 4.2.2)
    on ciphertexts: the oracle's chain DENSE, SQUARE, DENSE at N = 2048
    decrypts to the plaintext integer network mod t, and its slot-level run
    equals it too."""
    from oracle import network as nw
    p = wl.PARAMS["toy2048"]
    rs = wl.rng(21, 1)
    W1, W2 = rs.integers(-128, 128, (6, 8)), rs.integers(-128, 128, (4, 6))
    b1, b2 = rs.integers(-1000, 1000, 6), rs.integers(-1000, 1000, 4)
    ol = [("dense", W1, b1), ("square",), ("dense", W2, b2)]
    x = rs.integers(-128, 128, 8)
    exp = list(nw._mod(nw.dense_chain_plain(x, ol), p.t))
    assert exp == [int(v) % p.t for v in (W2.dot((W1.dot(x) + b1) ** 2) + b2)]
    sched = nw.dense_chain_schedule(ol, p.N, sparse)
    ins = nw.dense_chain_inputs(x, p.N, sparse)
    slots, _ = nw.run_slots(sched, ins, p.t)
    octx = bfv.Context(p)
    keys = bfv.keygen(octx, 5, nw.galois_elements(sched))
    cts = [bfv.encrypt(octx, keys, bfv.encode(octx, nw.dense_slots(m, p.N, p.t)), 6, i) for i, m in enumerate(ins)]
    outs, _ = nw.run_ciphertexts(octx, keys, sched, cts)
    dec = [bfv.decode(octx, bfv.decrypt(octx, keys, o)) for o in outs]
    if not sparse:   # dense input: row major, then column major last: one dense message
        assert [int(dec[0][j]) for j in range(4)] == exp and [int(slots[0][j]) for j in range(4)] == exp
        assert not np.any(dec[0][4:]) and len(outs) == 1
    else:            # sparse input: column major, then row major last: every slot of message j holds y_j
        assert [int(d[0]) for d in dec] == exp and all(np.all(d == d[0]) for d in dec)
        assert [int(s[0]) for s in slots] == exp


@pytest.mark.parametrize("recipe", ["full", "shared"])
def test_conv_chain_schedule_equals_plain_network(recipe):
    """The MNIST front end followed by a longer chain (DENSE 845 -> 24,
    SQUARE, DENSE 24 -> 12, SQUARE, DENSE 12 -> 10): the plain network with
    the MNIST layers is `mnist_plain`; the slot-level run of the oracle's
    schedule (stacked rounds, then dense vector - row major on the
    interleaved vector, then sparse vector - column major) gives the plain
    network mod t at slots 0..9 of its one output message, under both
    reductions of the first dense layer."""
    from oracle import network as nw
    wts, img = wl.mnist_weights(), wl.mnist_image(index=2)
    mn = [("dense", wts.w1, wts.b1), ("square",), ("dense", wts.w2, wts.b2)]
    assert list(nw.conv_chain_plain(img, wts.conv_w, wts.conv_b, mn)) == list(nw.mnist_plain(img, wts))
    rs = wl.rng(22, 1)
    W1, W2, W3 = rs.integers(-128, 128, (24, 845)), rs.integers(-128, 128, (12, 24)), rs.integers(-128, 128, (10, 12))
    b1, b2, b3 = rs.integers(-1000, 1000, 24), rs.integers(-1000, 1000, 12), rs.integers(-1000, 1000, 10)
    ol = [("dense", W1, b1), ("square",), ("dense", W2, b2), ("square",), ("dense", W3, b3)]
    t = 1146881
    exp = list(nw._mod(nw.conv_chain_plain(img, wts.conv_w, wts.conv_b, ol), t))
    sched = nw.conv_chain_schedule(wts.conv_w, wts.conv_b, ol, 16384, recipe)
    outs, _ = nw.run_slots(sched, nw.mnist_inputs(img), t)
    assert len(outs) == 1 and [int(outs[0][j]) for j in range(10)] == exp
    assert sched.out_slots == [{j: f"y{j}" for j in range(10)}]
    # 12 rows of the row-major layer, each summed over the whole message
    assert sum(1 for op in sched.ops if op[0] == "rotate" and op[3] == nw.ROW_SWAP) == 1 + 12


def test_cifar_chain_schedule_equals_plain_network():
    """The CIFAR-shaped front end followed by a chain: with the tail SQUARE,
    DENSE the plain network is `cifar_plain`; with SQUARE, DENSE H -> 6,
    SQUARE, DENSE 6 -> 10 the slot-level run of the oracle's schedule (dense
    vector - row major on the second convolution's dense output, then sparse
    vector - column major) equals the plain network mod t at slots 0..9."""
    from oracle import network as nw
    w = wl.cifar_weights(m1=5, m2=3, v2=1)
    img = wl.cifar_image(index=1)[:, :16, :16]
    pad = nw.cifar_padded(img)
    assert list(nw.cifar_chain_plain(pad, w, [("square",), ("dense", w.w3, w.b3)])) == list(nw.cifar_plain(pad, w))
    rs = wl.rng(24, 1)
    W1, b1 = rs.integers(-128, 128, (6, 3)), rs.integers(-1000, 1000, 6)
    W2, b2 = rs.integers(-128, 128, (10, 6)), rs.integers(-1000, 1000, 10)
    tail = [("square",), ("dense", W1, b1), ("square",), ("dense", W2, b2)]
    t = 1146881
    exp = list(nw._mod(nw.cifar_chain_plain(pad, w, tail), t))
    sched = nw.cifar_chain_schedule(w, tail, 18)
    outs, _ = nw.run_slots(sched, nw.cifar_inputs(pad), t)
    assert len(outs) == 1 and [int(outs[0][j]) for j in range(10)] == exp


@pytest.mark.parametrize("recipe", ["full", "shared"])
def test_hoisted_sums_schedule_equals_plain_network(recipe):
    """The hoisted form of the MNIST schedule's sums (groups of up to three
    rotate-and-sum steps as hoisted rotations by their subset sums, shifted
    combinations in one level) gives the plain network at the valid slots,
    as the sequential form does, with more rotations in fewer levels of key
    switches."""
    from oracle import network as nw
    wts, img = wl.mnist_weights(), wl.mnist_image(index=6)
    t = 1146881
    exp = list(nw._mod(nw.mnist_plain(img, wts), t))
    seq = nw.mnist_schedule(wts, recipe=recipe)
    hoi = nw.mnist_schedule(wts, recipe=recipe, sums="hoisted")
    outs, _ = nw.run_slots(hoi, nw.mnist_inputs(img), t)
    got = [int(o[0]) for o in outs] if recipe == "full" else [int(outs[0][8 * o]) for o in range(10)]
    assert got == exp
    assert hoi.count("rotate") > seq.count("rotate") and hoi.count("rotate_hoisted") > seq.count("rotate_hoisted")

    def depth(sc):
        # longest chain of key switches (rotations and squares) through the ops
        d = {}
        for op in sc.ops:
            srcs = [op[2], op[3]] if op[0] == "add" else [op[2]]
            base = max((d.get(x, 0) for x in srcs), default=0)
            d[op[1]] = base + (1 if op[0] in ("rotate", "rotate_hoisted", "square") else 0)
        return max(d[o] for o in sc.outputs)
    assert depth(hoi) < depth(seq)
