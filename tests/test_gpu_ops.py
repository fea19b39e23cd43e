"""GPU parity: every library operation against the oracle, word for word, in
coefficient form, on the same seeded inputs (N = 1024 to 16384)."""
import numpy as np
import pytest

from oracle import bfv
from paper_1812_10659_amd import workloads as wl

pytestmark = pytest.mark.gpu

# the last four: key-switching digits of two primes with two special primes
# (one ciphertext prime, three, seven and twelve)
PSETS = ["toy1024", "toy2048", "n4096_3q", "n8192", "mnist_n16384", "l12_n16384", "toy1024_l1_k2", "toy1024_k2",
         "mnist_n16384_k2", "l12_n16384_k2"]
STEPS = [1, -1, 7, bfv.ROW_SWAP]
SEED = 0x5EED_0001


def _u32(t):
    from paper_1812_10659_amd import lola
    return lola.to_numpy_u32(t)


def _up(ctx, limbs):
    """oracle coefficient-form ciphertext -> device NTT form"""
    from paper_1812_10659_amd import lola
    arr = np.stack([np.asarray(c, dtype=np.uint64) for c in limbs]).astype(np.uint32)
    return ctx.from_coeff(lola.from_numpy_u32(arr, ctx.device))


def _down(ctx, ct):
    return _u32(ctx.to_coeff(ct)).astype(np.uint64)


def _bitrev(k, bits):
    return int(format(k, f"0{bits}b")[::-1], 2)


@pytest.fixture(scope="module", params=PSETS)
def env(request):
    import torch
    from paper_1812_10659_amd import lola
    p = wl.PARAMS[request.param]
    print(f"[gpu-ops] params {p.name} N={p.N} L={p.L}", flush=True)
    ctx = lola.Context(p)
    octx = bfv.Context(p)
    gal = [bfv.galois_element(p.N, s) for s in STEPS]
    okeys = bfv.keygen(octx, SEED, gal)
    sk = ctx.keygen_secret(SEED)
    pk = ctx.keygen_public(SEED, sk)
    rlk = ctx.keygen_switch(SEED, sk, 0)
    gks = {g: ctx.keygen_switch(SEED, sk, g) for g in gal}
    torch.cuda.synchronize()
    rs = np.random.default_rng(p.N)
    m1 = rs.integers(0, p.t, p.N).astype(np.uint64)
    m2 = rs.integers(0, p.t, p.N).astype(np.uint64)
    c1 = bfv.encrypt(octx, okeys, m1, 11, 1)
    c2 = bfv.encrypt(octx, okeys, m2, 11, 2)
    return dict(p=p, ctx=ctx, octx=octx, okeys=okeys, sk=sk, pk=pk, rlk=rlk, gks=gks, gal=gal,
                m=(m1, m2), c=(c1, c2))


def test_galois_elements_agree(env):
    from paper_1812_10659_amd import lola
    N = env["p"].N
    for s in STEPS + [0, 3, -5, N // 2 - 1]:
        assert lola.galois_element(N, s) == bfv.galois_element(N, s)


def test_ntt_is_evaluation_at_odd_powers(env):
    from paper_1812_10659_amd import lola
    ctx, p = env["ctx"], env["p"]
    primes = list(p.q) + list(p.special) + [None] * ctx.n_aux + [p.t]
    idx = [i for i in range(len(primes)) if primes[i] is not None]
    rs = np.random.default_rng(1)
    x = np.stack([rs.integers(0, primes[i], p.N) for i in idx]).astype(np.uint32)
    xd = lola.from_numpy_u32(x, ctx.device)
    y = _u32(ctx.ntt_limbs(xd, idx))
    bits = p.N.bit_length() - 1
    br = np.array([_bitrev(k, bits) for k in range(p.N)])
    for row, i in enumerate(idx):
        m = primes[i]
        ev = np.empty(p.N, np.uint64)
        bfv.lib().or_eval_odd(x[row].astype(np.uint64), ev, p.N, m, bfv.min_root_2n(m, p.N))
        assert np.array_equal(y[row].astype(np.uint64), ev[br]), f"prime index {i}"
    back = _u32(ctx.ntt_limbs(lola.from_numpy_u32(y, ctx.device), idx, inverse=True))
    assert np.array_equal(back, x)


def _ntt_case(env):
    """Five limbs (first and last data prime, P, t, first prime again: an odd
    count, so the last workgroup of the 2- and 4-limb tiles is partial) with
    the oracle's evaluation at odd powers of the minimal root, bit-reversed."""
    from paper_1812_10659_amd import lola
    ctx, p = env["ctx"], env["p"]
    primes = list(p.q) + list(p.special) + [None] * ctx.n_aux + [p.t]
    idx = [0, p.L - 1, p.L, len(primes) - 1, 0]
    rs = np.random.default_rng(7)
    x = np.stack([rs.integers(0, primes[i], p.N) for i in idx]).astype(np.uint32)
    bits = p.N.bit_length() - 1
    br = np.array([_bitrev(k, bits) for k in range(p.N)])
    exp = []
    for row, i in enumerate(idx):
        ev = np.empty(p.N, np.uint64)
        bfv.lib().or_eval_odd(x[row].astype(np.uint64), ev, p.N, primes[i], bfv.min_root_2n(primes[i], p.N))
        exp.append(ev[br])
    return idx, x, lola.from_numpy_u32(x, ctx.device), np.stack(exp)


def test_ntt_cyclic_limbs_equal_the_descriptor_path(env):
    """Limbs under primes 0, 1, .., L-1, 0, 1, .. (consecutive polynomials,
    with a ragged last one) launch without descriptors; the same limbs in
    reverse order go through descriptors.  Both directions agree word for
    word."""
    import torch
    from paper_1812_10659_amd import lola
    ctx, p = env["ctx"], env["p"]
    L = p.L
    n = 3 * L + 2
    idx = np.arange(n, dtype=np.uint32) % L
    rs = np.random.default_rng(5)
    x = np.stack([rs.integers(0, p.q[i], p.N) for i in idx]).astype(np.uint32)
    xd = lola.from_numpy_u32(x, ctx.device)
    xr = lola.from_numpy_u32(np.ascontiguousarray(x[::-1]), ctx.device)
    for inverse in (False, True):
        y1 = _u32(ctx.ntt_limbs(xd, idx, inverse=inverse))
        y2 = _u32(ctx.ntt_limbs(xr, np.ascontiguousarray(idx[::-1]), inverse=inverse))
        assert np.array_equal(y1, y2[::-1]), inverse
    torch.cuda.synchronize()


def test_every_ntt_variant_is_evaluation_at_odd_powers(env):
    """Every compiled batched-NTT variant (radix split x limbs per workgroup)
    gives the oracle's evaluation and inverts exactly."""
    from paper_1812_10659_amd import lola
    ctx = env["ctx"]
    idx, x, xd, exp = _ntt_case(env)
    variants = ctx.ntt_variants()
    assert variants[0][1] == 1 and len(variants) >= 12
    try:
        for v, (split, lpw) in enumerate(variants):
            ctx.ntt_set_variant(v)
            y = _u32(ctx.ntt_limbs(xd, idx))
            assert np.array_equal(y.astype(np.uint64), exp), f"variant {split}/{lpw}"
            back = _u32(ctx.ntt_limbs(lola.from_numpy_u32(y, ctx.device), idx, inverse=True))
            assert np.array_equal(back, x), f"variant {split}/{lpw} inverse"
    finally:
        ctx.ntt_set_variant(0)


def test_ntt_autotune_picks_fastest_and_keeps_results(env):
    ctx = env["ctx"]
    idx, x, xd, exp = _ntt_case(env)
    try:
        chosen, table = ctx.ntt_autotune(n_limbs=2 * env["p"].L + 3, reps=2)
        assert ctx.ntt_variant() == chosen and len(table) == len(ctx.ntt_variants())
        ms = [t[2] for t in table]
        assert all(m > 0 for m in ms) and ms[chosen] == min(ms)
        assert np.array_equal(_u32(ctx.ntt_limbs(xd, idx)).astype(np.uint64), exp)
    finally:
        ctx.ntt_set_variant(0)


def test_keys_match_oracle(env):
    ctx, octx, ok = env["ctx"], env["octx"], env["okeys"]
    s_res = octx.small_to_limbs(ok.sk.s, octx.moduli)
    assert np.array_equal(_u32(ctx.export_sk(env["sk"])).astype(np.uint64), s_res)
    pk = _u32(ctx.export_pk(env["pk"])).astype(np.uint64)
    assert np.array_equal(pk[0], ok.pk0) and np.array_equal(pk[1], ok.pk1)
    for key, ref in [(env["rlk"], ok.rlk)] + [(env["gks"][g], ok.galois[g]) for g in env["gal"][:2]]:
        k = _u32(ctx.export_ksk(key)).astype(np.uint64)   # [dn][2][L+K][N]
        assert np.array_equal(k[:, 0], ref.b) and np.array_equal(k[:, 1], ref.a)


def test_encode_decode_match_oracle(env):
    ctx, octx, p = env["ctx"], env["octx"], env["p"]
    v = np.random.default_rng(2).integers(-3 * p.t, 3 * p.t, p.N)
    pt = ctx.encode(v)
    assert np.array_equal(_u32(pt).astype(np.uint64), bfv.encode(octx, v))
    assert np.array_equal(ctx.decode(pt), np.mod(v, p.t))


def test_encrypt_matches_oracle(env):
    ctx, octx, p = env["ctx"], env["octx"], env["p"]
    m = env["m"][0]
    from paper_1812_10659_amd import lola
    pt = lola.from_numpy_u32(m.astype(np.uint32), ctx.device)
    ct = ctx.encrypt(env["pk"], pt, 11, 1)
    got = _down(ctx, ct)
    assert np.array_equal(got[0], env["c"][0][0]) and np.array_equal(got[1], env["c"][0][1])


def test_decrypt_matches_oracle(env):
    ctx, octx = env["ctx"], env["octx"]
    c1, c2 = env["c"]
    d = _u32(ctx.decrypt(env["sk"], _up(ctx, c1))).astype(np.uint64)
    assert np.array_equal(d, bfv.decrypt(octx, env["okeys"], c1))
    assert np.array_equal(d, env["m"][0])
    c3 = bfv.mul(octx, c1, c2)
    d3 = _u32(ctx.decrypt(env["sk"], _up(ctx, c3))).astype(np.uint64)
    assert np.array_equal(d3, bfv.decrypt(octx, env["okeys"], c3))


def test_client_batches_match_oracle_and_single_calls(env):
    """Batched encode / decode / encrypt / decrypt: every message equals the
    single call word for word, across the scratch chunks (64 messages for the
    codec, 16 for encryption), and sampled messages equal the oracle."""
    import torch
    from paper_1812_10659_amd import lola
    ctx, octx, p = env["ctx"], env["octx"], env["p"]
    rs = np.random.default_rng(7)
    v = rs.integers(-3 * p.t, 3 * p.t, (70, p.N))
    pts = ctx.encode_batch(v)
    for i in (0, 63, 64, 69):
        assert np.array_equal(_u32(pts[i]).astype(np.uint64), bfv.encode(octx, v[i])), i
    for i in range(70):
        assert torch.equal(pts[i], ctx.encode(v[i])), i
    assert np.array_equal(ctx.decode_batch(pts).cpu().numpy(), np.mod(v, p.t))

    n = 19
    m = rs.integers(0, p.t, (n, p.N)).astype(np.uint64)
    m[0] = env["m"][0]
    mp = lola.from_numpy_u32(m.astype(np.uint32), ctx.device)
    cts = ctx.encrypt_batch(env["pk"], mp, 11, 1)
    got = _down(ctx, cts[0])
    assert np.array_equal(got[0], env["c"][0][0]) and np.array_equal(got[1], env["c"][0][1])
    ref = bfv.encrypt(octx, env["okeys"], m[17], 11, 18)
    got = _down(ctx, cts[17])
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    for i in range(n):
        assert torch.equal(cts[i], ctx.encrypt(env["pk"], mp[i], 11, 1 + i)), i
    assert np.array_equal(_u32(ctx.decrypt_batch(env["sk"], cts)).astype(np.uint64), m)

    # size-3 ciphertexts (products before relinearization)
    c3 = torch.stack([ctx.mul(cts[i], cts[i + 1]) for i in range(3)])
    d3 = ctx.decrypt_batch(env["sk"], c3)
    for i in range(3):
        assert torch.equal(d3[i], ctx.decrypt(env["sk"], c3[i])), i
    prod = bfv.mul(octx, list(_down(ctx, cts[1])), list(_down(ctx, cts[2])))
    assert np.array_equal(_u32(d3[1]).astype(np.uint64), bfv.decrypt(octx, env["okeys"], prod))
    # empty batches are no-ops; object ids past 2^32 are refused
    ctx.encode_batch(np.zeros((0, p.N), dtype=np.int64))
    ctx.encrypt_batch(env["pk"], mp[:0], 11, 1)
    with pytest.raises(lola.LolaError):
        ctx.encrypt_batch(env["pk"], mp[:3], 11, (1 << 32) - 2)
    torch.cuda.synchronize()


def test_linear_ops_match_oracle(env):
    from paper_1812_10659_amd import lola
    ctx, octx, p = env["ctx"], env["octx"], env["p"]
    c1, c2 = env["c"]
    m2 = env["m"][1]
    a, b = _up(ctx, c1), _up(ctx, c2)
    pt = lola.from_numpy_u32(m2.astype(np.uint32), ctx.device)
    assert np.array_equal(_down(ctx, ctx.add(a, b)), np.stack(bfv.add(octx, c1, c2)))
    assert np.array_equal(_down(ctx, ctx.add_plain(a, ctx.plain_add_form(pt))), np.stack(bfv.add_plain(octx, c1, m2)))
    assert np.array_equal(_down(ctx, ctx.mul_plain(a, ctx.plain_mul_form(pt))), np.stack(bfv.mul_plain(octx, c1, m2)))
    for w in (0, 1, -1, 127, -128, p.t - 1, p.t // 2, p.t // 2 + 1, 10**12 + 7):
        assert np.array_equal(_down(ctx, ctx.mul_scalar(a, w)), np.stack(bfv.mul_scalar(octx, c1, w))), w
    # in place
    x = _up(ctx, c1)
    ctx.add(x, b, out=x)
    assert np.array_equal(_down(ctx, x), np.stack(bfv.add(octx, c1, c2)))


def test_mul_matches_oracle(env):
    ctx, octx = env["ctx"], env["octx"]
    c1, c2 = env["c"]
    got = _down(ctx, ctx.mul(_up(ctx, c1), _up(ctx, c2)))
    assert np.array_equal(got, np.stack(bfv.mul(octx, c1, c2)))
    got = _down(ctx, ctx.mul(_up(ctx, c1), _up(ctx, c1)))
    assert np.array_equal(got, np.stack(bfv.mul(octx, c1, c1)))
    # a square from one buffer transforms and extends its operand once
    x = _up(ctx, c2)
    assert np.array_equal(_down(ctx, ctx.mul(x, x)), np.stack(bfv.mul(octx, c2, c2)))


def test_mul_batch_mixes_squares_and_products(env):
    """One batched launch with products of two buffers and squares of one."""
    from paper_1812_10659_amd import batched
    ctx, octx = env["ctx"], env["octx"]
    c1, c2 = env["c"]
    x1, x2 = _up(ctx, c1), _up(ctx, c2)
    a, b = [x1, x2, x1, x2], [x2, x2, x1, x1]
    outs = [ctx.empty_ct(3) for _ in a]
    batched.mul_batch(ctx, a, b, outs)
    refs = [bfv.mul(octx, c1, c2), bfv.mul(octx, c2, c2), bfv.mul(octx, c1, c1), bfv.mul(octx, c2, c1)]
    for k, (o, r) in enumerate(zip(outs, refs)):
        assert np.array_equal(_down(ctx, o), np.stack(r)), f"pair {k}"


def test_relin_matches_oracle(env):
    ctx, octx = env["ctx"], env["octx"]
    c1, c2 = env["c"]
    c3 = bfv.mul(octx, c1, c2)
    got = _down(ctx, ctx.relin(env["rlk"], _up(ctx, c3)))
    assert np.array_equal(got, np.stack(bfv.relin(octx, c3, env["okeys"].rlk)))


@pytest.mark.parametrize("step", STEPS, ids=str)
def test_rotate_matches_oracle(env, step):
    ctx, octx = env["ctx"], env["octx"]
    c1 = env["c"][0]
    g = bfv.galois_element(env["p"].N, step)
    got = _down(ctx, ctx.rotate(env["gks"][g], g, _up(ctx, c1)))
    assert np.array_equal(got, np.stack(bfv.rotate(octx, c1, step, env["okeys"])))


def test_keyswitch_batch_ragged(env):
    """Mixed rotations and a relinearisation in one batch (uneven keys)."""
    ctx, octx, ok = env["ctx"], env["octx"], env["okeys"]
    c1, c2 = env["c"]
    c3 = bfv.mul(octx, c1, c2)
    items, refs = [], []
    for k, step in enumerate([1, bfv.ROW_SWAP, -1, 7, 1]):
        src = c1 if k % 2 == 0 else c2
        g = bfv.galois_element(env["p"].N, step)
        items.append((_up(ctx, src), env["gks"][g], g))
        refs.append(bfv.rotate(octx, src, step, ok))
    items.append((_up(ctx, c3), env["rlk"], 0))
    refs.append(bfv.relin(octx, c3, ok.rlk))
    outs = ctx.keyswitch_batch(items)
    for o, r in zip(outs, refs):
        assert np.array_equal(_down(ctx, o), np.stack(r))


def test_rotate_hoisted_matches_oracle(env):
    """Rotations of one ciphertext sharing its decomposition: words equal the
    oracle's hoisted rotation; each decrypts like the plain rotation."""
    ctx, octx, ok = env["ctx"], env["octx"], env["okeys"]
    c1 = env["c"][0]
    gs = [bfv.galois_element(env["p"].N, s) for s in STEPS]
    outs = ctx.rotate_hoisted(_up(ctx, c1), gs, [env["gks"][g] for g in gs])
    for step, o in zip(STEPS, outs):
        ref = bfv.rotate_hoisted(octx, c1, step, ok)
        assert np.array_equal(_down(ctx, o), np.stack(ref)), f"step {step}"
        assert list(bfv.decrypt(octx, ok, ref)) == list(bfv.decrypt(octx, ok, bfv.rotate(octx, c1, step, ok)))


@pytest.mark.parametrize("n_jobs", [1, 4, 5, 16, 17, 40])
def test_keyswitch_both_inner_forms(env, n_jobs):
    """Launches of at most 16 jobs split the key inner product into one
    workgroup per (modulus, digit) term plus a fold; larger ones accumulate
    all digits per modulus.  Launches whose dn (L+K) terms per job fit one
    round of 256 workgroups compute the terms straight from the input and
    fold them inside the mod-down (two kernels).  All give the oracle's words
    (4 and 5 jobs sit on either side of the two-kernel form at L = 7 with one
    special prime, 16 and 17 on either side of the term split)."""
    ctx, octx, ok = env["ctx"], env["octx"], env["okeys"]
    c1, c2 = env["c"]
    c3 = bfv.mul(octx, c1, c2)
    base, refs = [], []
    for k, step in enumerate([1, bfv.ROW_SWAP, -1, 7]):
        src = c1 if k % 2 == 0 else c2
        g = bfv.galois_element(env["p"].N, step)
        base.append((_up(ctx, src), env["gks"][g], g))
        refs.append(bfv.rotate(octx, src, step, ok))
    base.append((_up(ctx, c3), env["rlk"], 0))
    refs.append(bfv.relin(octx, c3, ok.rlk))
    items = [base[k % len(base)] for k in range(n_jobs)]
    outs = ctx.keyswitch_batch(items)
    for k, o in enumerate(outs):
        assert np.array_equal(_down(ctx, o), np.stack(refs[k % len(base)])), f"job {k} of {n_jobs}"


def _ks_items(env, n_jobs=20):
    """n_jobs key switches (four rotations and a relinearisation, cycled) and
    their oracle results."""
    ctx, octx, ok = env["ctx"], env["octx"], env["okeys"]
    c1, c2 = env["c"]
    c3 = bfv.mul(octx, c1, c2)
    base, refs = [], []
    for k, step in enumerate([1, bfv.ROW_SWAP, -1, 7]):
        src = c1 if k % 2 == 0 else c2
        g = bfv.galois_element(env["p"].N, step)
        base.append((_up(ctx, src), env["gks"][g], g))
        refs.append(bfv.rotate(octx, src, step, ok))
    base.append((_up(ctx, c3), env["rlk"], 0))
    refs.append(bfv.relin(octx, c3, ok.rlk))
    return [base[k % len(base)] for k in range(n_jobs)], [refs[k % len(base)] for k in range(n_jobs)]


def test_every_ks_variant_gives_the_oracle_words(env):
    """Every compiled variant of each batched key-switch stage (radix split x
    LDS placement; several at N = 16384, one elsewhere), the other stages at
    their defaults, gives the oracle's words on a 20-job batch."""
    ctx = env["ctx"]
    items, refs = _ks_items(env)
    counts = [len(ctx.ks_variants(st)) for st in range(3)]
    assert counts == ([4, 3, 4] if env["p"].N == 16384 else [1, 1, 1])
    for st in range(3):
        for v in range(counts[st]):
            ctx.ks_set_variant(st, v)
            outs = ctx.keyswitch_batch(items)
            for k, o in enumerate(outs):
                assert np.array_equal(_down(ctx, o), np.stack(refs[k])), f"stage {st} variant {v} job {k}"
        ctx.ks_set_variant(st, 0)


def test_ks_autotune_keeps_the_words(env):
    """The key-switch autotuner times every variant (each checked against the
    default by the library), keeps the fastest per stage, and the batch
    afterwards still gives the oracle's words."""
    ctx = env["ctx"]
    items, refs = _ks_items(env)
    chosen, table = ctx.ks_autotune(n_jobs=24, reps=1)
    counts = [len(ctx.ks_variants(st)) for st in range(3)]
    assert len(table) == sum(counts) and all(ms > 0 for *_, ms in table)
    assert [ctx.ks_variant(st) for st in range(3)] == chosen
    for st in range(3):
        times = [ms for s, _, _, _, ms in table if s == st]
        # kept: no other variant is more than 1% faster than the chosen one
        assert min(times) >= 0.99 * times[chosen[st]] - 1e-6 or times[chosen[st]] == min(times)
    outs = ctx.keyswitch_batch(items)
    for k, o in enumerate(outs):
        assert np.array_equal(_down(ctx, o), np.stack(refs[k])), f"job {k} after autotuning"
    for st in range(3):
        ctx.ks_set_variant(st, 0)


def test_keys_and_encryption_with_256_bit_key(env):
    """Key words 2..7 set on the context (a full 256-bit ChaCha20 key): the
    secret, public and switching keys and an encryption equal the oracle's
    under the 256-bit seed; the words are reset afterwards."""
    from paper_1812_10659_amd import lola
    ctx, octx, p = env["ctx"], env["octx"], env["p"]
    words = [(0x9E3779B9 * (k + 3)) & 0xFFFFFFFF for k in range(6)]
    lo = 0x0123_4567_89AB_CDEF
    big = lo | sum(w << (64 + 32 * k) for k, w in enumerate(words))
    g = env["gal"][0]
    ok = bfv.keygen(octx, big, [g], relin=False)
    ctx.set_key_words(words)
    try:
        sk = ctx.keygen_secret(lo)
        pk = ctx.keygen_public(lo, sk)
        gk = ctx.keygen_switch(lo, sk, g)
        m = env["m"][1]
        ct = ctx.encrypt(pk, lola.from_numpy_u32(m.astype(np.uint32), ctx.device), lo ^ 0x55, 9)
    finally:
        ctx.set_key_words(None)
    assert np.array_equal(_u32(ctx.export_sk(sk)).astype(np.uint64), octx.small_to_limbs(ok.sk.s, octx.moduli))
    pkh = _u32(ctx.export_pk(pk)).astype(np.uint64)
    assert np.array_equal(pkh[0], ok.pk0) and np.array_equal(pkh[1], ok.pk1)
    k = _u32(ctx.export_ksk(gk)).astype(np.uint64)
    assert np.array_equal(k[:, 0], ok.galois[g].b) and np.array_equal(k[:, 1], ok.galois[g].a)
    oc = bfv.encrypt(octx, ok, m, (lo ^ 0x55) | (big >> 64 << 64), 9)
    got = _down(ctx, ct)
    assert np.array_equal(got[0], oc[0]) and np.array_equal(got[1], oc[1])
    # the same seed without the key words gives other keys
    assert not np.array_equal(_u32(ctx.export_sk(ctx.keygen_secret(lo))), _u32(ctx.export_sk(sk)))
