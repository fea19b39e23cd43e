"""GPU parity of whole networks: the compiled plan evaluated by the library
against the oracle's own schedule of the same recipes, ciphertext word for
word, and the decrypted results against the plaintext integer network mod t.
Also: batched requests equal single requests, and graph replays equal the
eager run."""
import numpy as np
import pytest

from oracle import bfv
from oracle import network as nw
from paper_1812_10659_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _setup(pname, layers, oracle_sched, values, key_seed, enc_seed, with_oracle=True, recipe=0, sums=0):
    import torch
    from paper_1812_10659_amd import lola, networks
    p = wl.PARAMS[pname]
    ctx = lola.Context(p)
    plan = lola.Plan(p, layers, recipe=recipe, sums=sums)
    plan.load(ctx)
    gal = plan.galois()
    sk = ctx.keygen_secret(key_seed)
    pk = ctx.keygen_public(key_seed, sk)
    rlk = ctx.keygen_switch(key_seed, sk, 0)
    gks = [ctx.keygen_switch(key_seed, sk, g) for g in gal]
    msgs = networks.pack_inputs(plan.input_map(), values)
    ins = [ctx.encrypt(pk, ctx.encode(m), enc_seed, i) for i, m in enumerate(msgs)]
    outs = [ctx.empty_ct() for _ in range(plan.info["n_outputs"])]
    req = dict(rlk=rlk, gks=gks, inputs=ins, outputs=outs)
    torch.cuda.synchronize()
    env = dict(p=p, ctx=ctx, plan=plan, sk=sk, req=req, msgs=msgs)
    if with_oracle:
        octx = bfv.Context(p)
        okeys = bfv.keygen(octx, key_seed, nw.galois_elements(oracle_sched))
        octs = [bfv.encrypt(octx, okeys, bfv.encode(octx, m), enc_seed, i) for i, m in enumerate(msgs)]
        env.update(octx=octx, okeys=okeys, octs=octs)
    return env


def _coeff(ctx, t):
    from paper_1812_10659_amd import lola
    return lola.to_numpy_u32(ctx.to_coeff(t)).astype(np.uint64)


def _decrypt_values(env):
    from paper_1812_10659_amd import networks
    ctx, plan = env["ctx"], env["plan"]
    slots = np.stack([ctx.decode(ctx.decrypt(env["sk"], o)) for o in env["req"]["outputs"]])
    return networks.unpack_outputs(plan.output_map(), slots)


def _run_and_compare(env, oracle_sched, expected):
    import torch
    ctx, plan = env["ctx"], env["plan"]
    plan.evaluate(ctx, [env["req"]])
    torch.cuda.synchronize()
    oouts, _ = nw.run_ciphertexts(env["octx"], env["okeys"], oracle_sched, env["octs"])
    for k, (g, o) in enumerate(zip(env["req"]["outputs"], oouts)):
        assert np.array_equal(_coeff(ctx, g), np.stack(o)), f"output {k} differs from the oracle"
    assert list(_decrypt_values(env)) == list(nw._mod(expected, env["p"].t))


def test_dense64_network_matches_oracle():
    from paper_1812_10659_amd import networks
    x, W = wl.dense64_inputs()
    print("[gpu-net] dense64", flush=True)
    sched = nw.dense64_schedule(W)
    env = _setup("n4096_3q", networks.dense64_layers(W), sched, x, wl.key_seed(0), wl.enc_seed(0))
    _run_and_compare(env, sched, nw.dense64_plain(x, W))


# (oracle recipe name, LOLA_RECIPE_*): the paper's layout and the shared reduction
RECIPES = [("full", 4), ("shared", 5)]


@pytest.mark.parametrize("name,recipe", RECIPES)
def test_mnist_network_matches_oracle(name, recipe):
    from paper_1812_10659_amd import networks
    w, img = wl.mnist_weights(), wl.mnist_image()
    print(f"[gpu-net] mnist {name}", flush=True)
    sched = nw.mnist_schedule(w, recipe=name)
    env = _setup("mnist_n16384", networks.mnist_layers(w), sched, networks.mnist_input_values(img),
                 wl.key_seed(1), wl.enc_seed(1), recipe=recipe)
    assert env["plan"].info["recipe"] == recipe
    _run_and_compare(env, sched, nw.mnist_plain(img, w))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("sums", ["sequential", "hoisted"])
def test_mnist_two_prime_digits_matches_oracle(sums):
    """The MNIST network with key-switching digits of two primes and two
    special primes (mnist_n16384_k2), shared reduction, in both forms of the
    sums: ciphertext words against the oracle's schedule run with the same
    key-switching reading, logits against the plain network."""
    from paper_1812_10659_amd import lola, networks
    w, img = wl.mnist_weights(), wl.mnist_image(index=5)
    print(f"[gpu-net] mnist, digits of two primes, {sums} sums", flush=True)
    sched = nw.mnist_schedule(w, recipe="shared", sums=sums)
    env = _setup("mnist_n16384_k2", networks.mnist_layers(w), sched, networks.mnist_input_values(img),
                 wl.key_seed(1) + 33, wl.enc_seed(1) + 33, recipe=lola.RECIPE_SHARED_REDUCTION,
                 sums=lola.SUMS_HOISTED if sums == "hoisted" else lola.SUMS_SEQUENTIAL)
    assert env["ctx"].K == 2 and env["ctx"].dnum == 4
    _run_and_compare(env, sched, nw.mnist_plain(img, w))


def test_mnist_hoisted_sums_matches_oracle():
    """The MNIST network in the layout for single requests (shared reduction,
    every rotate-and-sum and combination in the hoisted form: 106 rotations
    of which 93 hoisted, in fewer levels): words against the oracle's
    schedule in the same form, decrypted logits against the plain network;
    the batched evaluation of two requests equals their single runs."""
    import torch
    from paper_1812_10659_amd import lola, networks
    w, img = wl.mnist_weights(), wl.mnist_image(index=5)
    print("[gpu-net] mnist shared, hoisted sums", flush=True)
    sched = nw.mnist_schedule(w, recipe="shared", sums="hoisted")
    env = _setup("mnist_n16384", networks.mnist_layers(w), sched, networks.mnist_input_values(img),
                 wl.key_seed(1) + 21, wl.enc_seed(1) + 21, recipe=lola.RECIPE_SHARED_REDUCTION,
                 sums=lola.SUMS_HOISTED)
    assert env["plan"].info["sums"] == lola.SUMS_HOISTED and env["plan"].info["n_rotations"] == 106
    _run_and_compare(env, sched, nw.mnist_plain(img, w))
    ctx, plan, req = env["ctx"], env["plan"], env["req"]
    single = [_coeff(ctx, o) for o in req["outputs"]]
    twin = dict(req, outputs=[ctx.empty_ct() for _ in req["outputs"]])
    plan.evaluate(ctx, [req, twin])
    torch.cuda.synchronize()
    for a, b in zip(req["outputs"], twin["outputs"]):
        assert np.array_equal(_coeff(ctx, a), _coeff(ctx, b))
    assert all(np.array_equal(_coeff(ctx, o), s) for o, s in zip(req["outputs"], single))


@pytest.mark.parametrize("net", ["dense64", "small"])
def test_hoisted_sums_small_networks_match_oracle(net):
    """Dense-64 at N=4096 and LoLa-Small with hoisted sums: words against the
    oracle's schedules in the same form, outputs against the plain networks."""
    from paper_1812_10659_amd import lola, networks
    print(f"[gpu-net] {net}, hoisted sums", flush=True)
    if net == "dense64":
        x, W = wl.dense64_inputs()
        sched = nw.dense64_schedule(W, sums="hoisted")
        env = _setup("n4096_3q", networks.dense64_layers(W), sched, x, wl.key_seed(0) + 23, wl.enc_seed(0) + 23,
                     sums=lola.SUMS_HOISTED)
        _run_and_compare(env, sched, nw.dense64_plain(x, W))
    else:
        w, img = wl.mnist_small_weights(), wl.mnist_image(index=7)
        sched = nw.mnist_small_schedule(w, sums="hoisted")
        env = _setup("mnist_n16384", networks.mnist_small_layers(w), sched, networks.mnist_input_values(img),
                     wl.key_seed(1) + 25, wl.enc_seed(1) + 25, sums=lola.SUMS_HOISTED)
        _run_and_compare(env, sched, nw.mnist_small_plain(img, w))
    assert env["plan"].info["sums"] == lola.SUMS_HOISTED


@pytest.mark.timeout(600)
@pytest.mark.parametrize("net", ["dense_input", "head", "head_stacked"])
def test_hoisted_sums_larger_networks_match_oracle(net):
    """Hoisted sums on LoLa-Dense (shared reduction, eight data primes) and on
    the transfer head with 8 hidden units under both recipes: words against
    the oracle's schedules in the same form, outputs against the plain
    networks."""
    from paper_1812_10659_amd import lola, networks
    print(f"[gpu-net] {net}, hoisted sums", flush=True)
    H = lola.SUMS_HOISTED
    if net == "dense_input":
        w, img = wl.mnist_weights(), wl.mnist_image(index=9)
        sched = nw.mnist_dense_schedule(w, recipe="shared", sums="hoisted")
        env = _setup("mnist_dense_n16384", networks.mnist_dense_layers(w), sched, networks.mnist_input_values(img),
                     wl.key_seed(1) + 27, wl.enc_seed(1) + 27, recipe=lola.RECIPE_SHARED_REDUCTION, sums=H)
        _run_and_compare(env, sched, nw.mnist_plain(img, w))
    else:
        w = wl.head_weights()
        wt = wl.HeadWeights(w.w1[:8], w.b1[:8], w.w2[:, :8], w.b2)
        if net == "head":
            f = wl.head_features(4)
            sched = nw.head_schedule(w, n_hidden=8, sums="hoisted")
            env = _setup("head_n16384", networks.head_layers(w, 8), sched, f, wl.key_seed(3) + 29, wl.enc_seed(3) + 29,
                         recipe=lola.RECIPE_DENSE_ROW_MAJOR, sums=H)
            _run_and_compare(env, sched, np.concatenate([nw.head_plain(f[q], wt) for q in range(4)]))
        else:
            f = wl.head_features(1)
            sched = nw.head_stacked_schedule(w, n_hidden=8, sums="hoisted")
            env = _setup("head_n16384", networks.head_layers(w, 8), sched, f[0], wl.key_seed(3) + 31,
                         wl.enc_seed(3) + 31, recipe=lola.RECIPE_STACKED_ROW_MAJOR, sums=H)
            _run_and_compare(env, sched, nw.head_plain(f[0], wt))
    assert env["plan"].info["sums"] == H


@pytest.mark.timeout(600)
@pytest.mark.parametrize("net", ["dense_input", "head", "head_stacked"])
def test_two_prime_digits_other_networks_match_oracle(net):
    """Key-switching digits of two primes with two special primes on
    LoLa-Dense (eight data primes: four digits) and on the transfer head with
    8 hidden units under both recipes (six data primes: three digits): words
    against the oracle's schedules run with the same reading, outputs
    against the plain networks."""
    from paper_1812_10659_amd import lola, networks
    print(f"[gpu-net] {net}, digits of two primes", flush=True)
    if net == "dense_input":
        w, img = wl.mnist_weights(), wl.mnist_image(index=11)
        sched = nw.mnist_dense_schedule(w, recipe="shared")
        env = _setup("mnist_dense_n16384_k2", networks.mnist_dense_layers(w), sched,
                     networks.mnist_input_values(img), wl.key_seed(1) + 37, wl.enc_seed(1) + 37,
                     recipe=lola.RECIPE_SHARED_REDUCTION)
        _run_and_compare(env, sched, nw.mnist_plain(img, w))
    else:
        w = wl.head_weights()
        wt = wl.HeadWeights(w.w1[:8], w.b1[:8], w.w2[:, :8], w.b2)
        if net == "head":
            f = wl.head_features(4)
            sched = nw.head_schedule(w, n_hidden=8)
            env = _setup("head_n16384_k2", networks.head_layers(w, 8), sched, f, wl.key_seed(3) + 39,
                         wl.enc_seed(3) + 39, recipe=lola.RECIPE_DENSE_ROW_MAJOR)
            _run_and_compare(env, sched, np.concatenate([nw.head_plain(f[q], wt) for q in range(4)]))
        else:
            f = wl.head_features(1)
            sched = nw.head_stacked_schedule(w, n_hidden=8)
            env = _setup("head_n16384_k2", networks.head_layers(w, 8), sched, f[0], wl.key_seed(3) + 41,
                         wl.enc_seed(3) + 41, recipe=lola.RECIPE_STACKED_ROW_MAJOR)
            _run_and_compare(env, sched, nw.head_plain(f[0], wt))
    assert env["ctx"].K == 2


@pytest.mark.parametrize("name,recipe", RECIPES)
def test_mnist_dense_input_network_matches_oracle(name, recipe):
    """LoLa-Dense: one dense input message, masks and rotations build the
    convolution messages; eight data primes."""
    from paper_1812_10659_amd import networks
    w, img = wl.mnist_weights(), wl.mnist_image(index=2)
    print(f"[gpu-net] mnist dense input {name}", flush=True)
    sched = nw.mnist_dense_schedule(w, recipe=name)
    env = _setup("mnist_dense_n16384", networks.mnist_dense_layers(w), sched, networks.mnist_input_values(img),
                 wl.key_seed(1) + 9, wl.enc_seed(1) + 9, recipe=recipe)
    assert env["plan"].info["recipe"] == recipe
    _run_and_compare(env, sched, nw.mnist_plain(img, w))


@pytest.mark.timeout(600)
def test_conv_then_dense_chain_matches_oracle():
    """A convolution network with a longer dense chain, which no fixed
    pattern covers: CONV2D, SQUARE, DENSE 845 -> 16, SQUARE, DENSE 16 -> 12,
    SQUARE, DENSE 12 -> 10 (the first dense layer in stacked rounds with the
    shared reduction, then dense vector - row major on the interleaved
    vector and sparse vector - column major on its sparse result; ten data
    primes): words against the oracle's schedule of the same network, and
    the decrypted outputs against the plain network."""
    from paper_1812_10659_amd import lola, networks
    w, img = wl.mnist_weights(), wl.mnist_image(index=3)
    rs = wl.rng(23, 1)
    dims = [845, 16, 12, 10]
    layers = [lola.conv2d(w.conv_w, w.conv_b, networks.MNIST_PAD, 2), lola.square()]
    ol = []
    for i in range(len(dims) - 1):
        W = rs.integers(-128, 128, (dims[i + 1], dims[i]))
        b = rs.integers(-1000, 1000, dims[i + 1])
        if i:
            layers.append(lola.square())
            ol.append(("square",))
        layers.append(lola.dense(W, b))
        ol.append(("dense", W, b))
    print("[gpu-net] convolution then a dense chain", flush=True)
    sched = nw.conv_chain_schedule(w.conv_w, w.conv_b, ol, 16384, "shared")
    env = _setup("chain_n16384", layers, sched, networks.mnist_input_values(img), wl.key_seed(1) + 13,
                 wl.enc_seed(1) + 13, recipe=lola.RECIPE_SHARED_REDUCTION)
    assert env["plan"].info["recipe"] == lola.RECIPE_SHARED_REDUCTION
    _run_and_compare(env, sched, nw.conv_chain_plain(img, w.conv_w, w.conv_b, ol))


@pytest.mark.timeout(600)
def test_two_convolutions_then_dense_chain_matches_oracle():
    """Two convolutions followed by two dense layers (CONV2D, SQUARE, CONV2D,
    SQUARE, DENSE 3 -> 6, SQUARE, DENSE 6 -> 10; the CIFAR-shaped front end
    on a 3x16x16 image with 5 and 3 maps, ten data primes): words against
    the oracle's schedule, and the decrypted outputs against the plain
    network."""
    from paper_1812_10659_amd import lola, networks
    w = wl.cifar_weights(m1=5, m2=3, v2=1)
    img = wl.cifar_image(index=2)[:, :16, :16]
    rs = wl.rng(25, 1)
    W1, b1 = rs.integers(-128, 128, (6, 3)), rs.integers(-1000, 1000, 6)
    W2, b2 = rs.integers(-128, 128, (10, 6)), rs.integers(-1000, 1000, 10)
    tail = [("square",), ("dense", W1, b1), ("square",), ("dense", W2, b2)]
    layers = networks.cifar_layers(w, 18)[:3] + [lola.square(), lola.dense(W1, b1), lola.square(),
                                                 lola.dense(W2, b2)]
    print("[gpu-net] two convolutions then a dense chain", flush=True)
    sched = nw.cifar_chain_schedule(w, tail, 18)
    env = _setup("chain_n16384", layers, sched, networks.cifar_input_values(img), wl.key_seed(1) + 17,
                 wl.enc_seed(1) + 17)
    _run_and_compare(env, sched, nw.cifar_chain_plain(nw.cifar_padded(img), w, tail))


@pytest.mark.parametrize("pname", ["cifar_n16384", "cifar_n16384_k2"])
def test_cifar_shaped_small_matches_oracle(pname):
    """The two-convolution recipe on a reduced case (3x16x16 image, 5 and 3
    maps), ciphertext words against the oracle's schedule, under both
    key-switching shapes."""
    from paper_1812_10659_amd import networks
    w = wl.cifar_weights(m1=5, m2=3, v2=1)
    img = wl.cifar_image(index=2)[:, :16, :16]
    print(f"[gpu-net] cifar-shaped, reduced, {pname}", flush=True)
    sched = nw.cifar_schedule(w, 18)
    env = _setup(pname, networks.cifar_layers(w, 18), sched, networks.cifar_input_values(img),
                 wl.key_seed(5), wl.enc_seed(5))
    _run_and_compare(env, sched, nw.cifar_plain(nw.cifar_padded(img), w))


def test_cifar_shaped_full_size_decrypts_to_network():
    """The full CIFAR-shaped network (83 and 163 maps, 57251 rotations) with
    the benchmark's parameter set (two-prime key-switching digits): the
    oracle's ciphertext run is far too slow, so the check is the decrypted
    logits against the plaintext network mod t."""
    import torch
    from paper_1812_10659_amd import networks
    w = wl.cifar_weights()
    img = wl.cifar_image(index=0)
    print("[gpu-net] cifar-shaped, full size", flush=True)
    env = _setup("cifar_n16384_k2", networks.cifar_layers(w), None, networks.cifar_input_values(img),
                 wl.key_seed(5) + 1, wl.enc_seed(5) + 1, with_oracle=False)
    env["plan"].evaluate(env["ctx"], [env["req"]])
    torch.cuda.synchronize()
    assert list(_decrypt_values(env)) == list(nw._mod(nw.cifar_plain(nw.cifar_padded(img), w), env["p"].t))


def test_mnist_small_network_matches_oracle():
    from paper_1812_10659_amd import networks
    w, img = wl.mnist_small_weights(), wl.mnist_image(index=3)
    print("[gpu-net] mnist small", flush=True)
    sched = nw.mnist_small_schedule(w)
    env = _setup("mnist_n16384", networks.mnist_small_layers(w), sched, networks.mnist_input_values(img),
                 wl.key_seed(1) + 5, wl.enc_seed(1) + 5)
    _run_and_compare(env, sched, nw.mnist_small_plain(img, w))


def test_head_network_truncated_matches_oracle():
    from paper_1812_10659_amd import networks
    w, f = wl.head_weights(), wl.head_features(4)
    print("[gpu-net] head, 8 hidden", flush=True)
    sched = nw.head_schedule(w, n_hidden=8)
    env = _setup("head_n16384", networks.head_layers(w, 8), sched, f, wl.key_seed(3), wl.enc_seed(3))
    wt = wl.HeadWeights(w.w1[:8], w.b1[:8], w.w2[:, :8], w.b2)
    _run_and_compare(env, sched, np.concatenate([nw.head_plain(f[q], wt) for q in range(4)]))


def test_head_stacked_recipe_truncated_matches_oracle():
    """The head compiled with the stacked vector - row major recipe (one
    query per message), ciphertext words against the oracle's schedule."""
    from paper_1812_10659_amd import lola, networks
    w, f = wl.head_weights(), wl.head_features(1)
    print("[gpu-net] head, stacked recipe, 8 hidden", flush=True)
    sched = nw.head_stacked_schedule(w, n_hidden=8)
    env = _setup("head_n16384", networks.head_layers(w, 8), sched, f[0], wl.key_seed(3) + 1, wl.enc_seed(3) + 1,
                 recipe=lola.RECIPE_STACKED_ROW_MAJOR)
    wt = wl.HeadWeights(w.w1[:8], w.b1[:8], w.w2[:, :8], w.b2)
    _run_and_compare(env, sched, nw.head_plain(f[0], wt))


@pytest.mark.timeout(900)
def test_head_network_full_size_matches_oracle():
    """Full 4096 -> 256 -> 10 head with 4 queries per ciphertext (dense vector
    - row major, 3407 rotations): ciphertext words against the oracle's
    schedule, and the decrypted results against the plaintext network."""
    from paper_1812_10659_amd import networks
    w, f = wl.head_weights(), wl.head_features(4)
    print("[gpu-net] head, full size, dense recipe (oracle: ~3400 rotations)", flush=True)
    sched = nw.head_schedule(w)
    env = _setup("head_n16384", networks.head_layers(w), sched, f, wl.key_seed(3), wl.enc_seed(3))
    expected = np.concatenate([nw.head_plain(f[q], w) for q in range(4)])
    _run_and_compare(env, sched, expected)


@pytest.mark.timeout(900)
def test_head_stacked_recipe_full_size_matches_oracle():
    """The full head compiled with the stacked vector - row major recipe (one
    query per message, 911 rotations), with the benchmark's parameter set
    (two-prime key-switching digits): ciphertext words against the oracle's
    schedule.  (The full dense row-major head above keeps one prime per
    digit, which the oracle runs faster.)"""
    from paper_1812_10659_amd import lola, networks
    w, f = wl.head_weights(), wl.head_features(1)
    print("[gpu-net] head, full size, stacked recipe, two-prime digits", flush=True)
    sched = nw.head_stacked_schedule(w)
    env = _setup("head_n16384_k2", networks.head_layers(w), sched, f[0], wl.key_seed(3) + 2, wl.enc_seed(3) + 2,
                 recipe=lola.RECIPE_STACKED_ROW_MAJOR)
    assert env["plan"].info["n_rotations"] == sched.count("rotate")
    _run_and_compare(env, sched, nw.head_plain(f[0], w))


@pytest.mark.parametrize("recipe,sparse", [(6, False), (7, True)])
def test_dense_chain_matches_oracle(recipe, sparse):
    """DENSE 64->32, SQUARE, DENSE 32->16, SQUARE, DENSE 16->10 on one query:
    dense vector - row major on dense inputs and sparse vector - column major
    on sparse ones (Sec. 4.2.2), ciphertext words against the oracle."""
    from paper_1812_10659_amd import lola
    rs = wl.rng(31, 3)
    dims = [64, 32, 16, 10]
    Ws = [rs.integers(-128, 128, (dims[i + 1], dims[i])) for i in range(3)]
    bs = [rs.integers(-1000, 1000, dims[i + 1]) for i in range(3)]
    layers = [lola.dense(Ws[0], bs[0]), lola.square(), lola.dense(Ws[1], bs[1]), lola.square(),
              lola.dense(Ws[2], bs[2])]
    ol = [("dense", Ws[0], bs[0]), ("square",), ("dense", Ws[1], bs[1]), ("square",), ("dense", Ws[2], bs[2])]
    x = rs.integers(-128, 128, 64)
    print(f"[gpu-net] dense chain, recipe {recipe}", flush=True)
    sched = nw.dense_chain_schedule(ol, 16384, sparse)
    env = _setup("mnist_n16384", layers, sched, x, wl.key_seed(6) + recipe, wl.enc_seed(6) + recipe, recipe=recipe)
    assert env["plan"].info["recipe"] == recipe
    _run_and_compare(env, sched, nw.dense_chain_plain(x, ol))


def test_batched_requests_equal_single_and_graph_replay():
    """Three requests with different keys and inputs in one evaluation equal
    three single evaluations; graph replays (with eager work in between)
    equal the eager result every time."""
    import torch
    from paper_1812_10659_amd import lola, networks
    _, W = wl.dense64_inputs()
    envs = []
    for k in range(3):
        x = wl.rng(1000 + k).integers(-128, 128, size=64)
        envs.append(_setup("n4096_3q", networks.dense64_layers(W), None, x, 77 + k, 99 + k, with_oracle=False))
    ctx, plan = envs[0]["ctx"], envs[0]["plan"]
    # re-home every request onto the first context (same parameters)
    reqs = []
    for e in envs:
        r = e["req"]
        reqs.append(dict(rlk=r["rlk"], gks=r["gks"], inputs=r["inputs"], outputs=[ctx.empty_ct() for _ in r["outputs"]]))
    plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    for e, r in zip(envs, reqs):
        e["plan"].evaluate(e["ctx"], [e["req"]])
        torch.cuda.synchronize()
        for a, b in zip(r["outputs"], e["req"]["outputs"]):
            assert torch.equal(a, b)
    eager = [[o.clone() for o in r["outputs"]] for r in reqs]
    s = torch.cuda.Stream()
    for rep in range(3):
        for r in reqs:
            for o in r["outputs"]:
                o.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            plan.evaluate(ctx, reqs, graph=True, stream=s)
        s.synchronize()
        junk = ctx.mul_scalar(reqs[0]["inputs"][0], 3)   # eager work between replays
        torch.cuda.synchronize()
        for r, ref in zip(reqs, eager):
            for a, b in zip(r["outputs"], ref):
                assert torch.equal(a, b), f"replay {rep}"
        del junk


def test_two_lane_batch_equals_single_requests():
    """A batch of 17 requests (two lanes of 9 and 8 on two streams) equals
    each request evaluated alone; so does the same batch as one lane (kernel
    timing on) and as graph replays captured with two lanes and with one,
    with eager runs between the replays."""
    import torch
    from paper_1812_10659_amd import lola, networks
    _, W = wl.dense64_inputs()
    envs = []
    for k in range(17):
        x = wl.rng(2000 + k).integers(-128, 128, size=64)
        envs.append(_setup("n4096_3q", networks.dense64_layers(W), None, x, 300 + k % 3, 400 + k, with_oracle=False))
    print("[gpu-net] two lanes, 17 requests", flush=True)
    ctx, plan = envs[0]["ctx"], envs[0]["plan"]
    reqs = [dict(rlk=e["req"]["rlk"], gks=e["req"]["gks"], inputs=e["req"]["inputs"],
                 outputs=[ctx.empty_ct() for _ in e["req"]["outputs"]]) for e in envs]
    singles = []
    for e in envs:
        e["plan"].evaluate(e["ctx"], [e["req"]])
        torch.cuda.synchronize()
        singles.append([o.clone() for o in e["req"]["outputs"]])

    def check(tag):
        for k, (r, ref) in enumerate(zip(reqs, singles)):
            for a, b in zip(r["outputs"], ref):
                assert torch.equal(a, b), f"{tag}: request {k}"
        for r in reqs:
            for o in r["outputs"]:
                o.zero_()
        torch.cuda.synchronize()

    plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    check("two lanes")
    lola.timing_enable(ctx, True)
    plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    lola.timing_enable(ctx, False)
    lola.kernel_timing(ctx)
    check("one lane")
    s = torch.cuda.Stream()

    def replay(tag):
        with torch.cuda.stream(s):
            plan.evaluate(ctx, reqs, graph=True, stream=s)
        s.synchronize()
        check(tag)

    replay("graph (two lanes captured)")
    plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    check("two lanes again")
    replay("graph replayed after eager work")
    plan.set_lanes(1)
    plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    check("lanes limited to one")
    replay("graph recaptured as one lane")
    replay("one-lane graph replayed")
    plan.set_lanes(2)
    replay("graph recaptured as two lanes")
