"""bench.py's own references, on the CPU: the plain networks its spot checks
compare decrypted results with must equal the oracle's plaintext networks, and
the algorithmic work and bytes of one key switch it reports are the stated
formulas; it refuses more than one GPU.  The oracle's per-operation timing
helper reports both thread settings and its labelled extrapolation."""
import os
import subprocess
import sys

import numpy as np

import bench
from oracle import network as nw
from oracle import crt as ocrt
from paper_1812_10659_amd import workloads as wl


def test_mnist_references_equal_the_oracle_networks():
    w = wl.mnist_weights()
    t = wl.PARAMS["mnist_n16384"].t
    for idx in (0, 3, 63):
        img = wl.mnist_image(index=idx)
        exact = nw.mnist_plain(img, w)
        assert [int(v) for v in bench._plain_logits_mod_t(img, w, t)] == [int(v) for v in nw._mod(exact, t)]
        assert [int(v) for v in bench._plain_logits_exact(img, w)] == [int(v) for v in exact]
    moduli = [p.t for p in wl.crt_params()]
    M = 1
    for m in moduli:
        M *= m
    assert 2 * ocrt.mnist_logit_bound(w) < M


def test_small_and_head_references_equal_the_oracle_networks():
    ws = wl.mnist_small_weights()
    img = wl.mnist_image(index=5)
    assert [int(v) for v in bench._plain_small_logits(img, ws)] == [int(v) for v in nw.mnist_small_plain(img, ws)]
    hw, f = wl.head_weights(), wl.head_features(2)
    for q in range(2):
        assert [int(v) for v in bench._head_plain(f[q], hw)] == [int(v) for v in nw.head_plain(f[q], hw)]


def test_cifar_reference_equals_the_oracle_network():
    w = wl.cifar_weights()
    t = wl.PARAMS["cifar_n16384"].t
    img = wl.cifar_image(index=0)
    exp = nw._mod(nw.cifar_plain(nw.cifar_padded(img), w), t)
    assert bench._cifar_plain_mod_t(img, w, t) == [int(v) for v in exp]


def test_reported_work_and_bytes_per_key_switch():
    N, L = 16384, 7
    # L^2 + 2 transforms (L - 1 for each of the L ciphertext primes, L for P,
    # two inverse transforms) of N/2 log2 N butterflies at 9 ops, and
    # 2 L (L+1) N multiply-accumulates at 7 ops
    assert bench.ks_inner_ops(N, L) == 9 * (L * L + 2) * (N // 2) * 14 + 7 * 2 * L * (L + 1) * N == 65486848
    # ciphertext in, key once, result out
    assert bench.ks_bytes(N, L) == 4 * N * (2 * L + 2 * L * (L + 1) + 2 * L) == 9175040
    assert np.isclose(bench.PEAK_VALU_LANE_OPS, 39.3216e12)
    # digits of two primes with two special primes, counted by hand at L = 7:
    # digits {0,1} {2,3} {4,5} {6}, nine target moduli.  Each ciphertext
    # prime's unit transforms the three digits that do not hold it (21), each
    # special prime's all four (8): 29 transforms, plus two inverse
    # transforms per special prime; 2 x 4 digits x 9 moduli key products; a
    # Garner step for every transformed pair whose digit has two primes: the
    # three two-prime digits times the seven moduli outside each (21)
    assert bench.ks_shape(L, 2) == (4, 9, 29, 21)
    by_hand = 9 * (29 + 4) * (N // 2) * 14 + 7 * 2 * 4 * 9 * N + 14 * 21 * N
    assert bench.ks_inner_ops(N, L, 2) == by_hand == 47136768
    assert bench.ks_bytes(N, L, 2) == 4 * N * (2 * L + 2 * 4 * 9 + 2 * L) == 6553600
    # one prime per digit is the same count at K = 1
    assert bench.ks_shape(L, 1) == (7, 8, 49, 0)


def test_oracle_per_op_times_and_their_extrapolation():
    r = bench.oracle_batch_ops()
    keys = [k for k in r if k.startswith("threads_")]
    from oracle import bfv
    assert "threads_1" in keys and len(keys) == len({bfv.max_threads(), 1})
    for k in keys:
        assert set(r[k]) == {"mul_plain_s", "mul_s", "relin_s", "rotate_s"} and all(v > 0 for v in r[k].values())
    a = r[max(keys, key=lambda k: int(k.split("_")[1]))]
    rot = int(wl.batch_rotation_counts(512).sum())
    est = 512 * a["mul_plain_s"] + 256 * (a["mul_s"] + a["relin_s"]) + rot * a["rotate_s"]
    assert abs(r["extrapolated_batch_s"] - round(est, 1)) < 0.11 and "extrapolated" in r["extrapolated_note"]


def test_bench_refuses_more_than_one_gpu():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""
