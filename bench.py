"""Benchmark: encrypted inferences/s of the MNIST-shaped LoLa network at N=16384.

One step = one batched evaluation of B encrypted requests (conv 5x5 s2, 5 maps
-> square -> dense 845->100 -> square -> dense 100->10), inputs already
encrypted and resident in HBM, every request's rotations, 24 plaintext
products, 125 scalar products and 2 squares run by the library.  The plan is
the compiler's default: of the two recipes for this network it keeps the
cheaper by its cost model, the shared reduction (58 rotations); the layout the
paper describes (154 rotations) is timed on the same batch as `paper_layout`.
Requests belong to `--clients` key sets (round robin), as a server holding
several clients' keys would see them.

The library runs a batch of 16 or more requests as two lanes (halves of the
batch on two streams, so each fills the other's launch tails).  The dominant
kernel's roofline (key-switch inner kernel) comes from a second pass of the
same steps with kernel timing on, which runs the batch as one lane so every
launch is timed alone with HIP events on its launch stream.

Also reported: single-request latency p50/p99 (the unbatched path), NTT and
key-switch HBM throughput on algorithmic bytes, and the CPU oracle on the host
cores.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock = 39.3e12 /s
PEAK_HBM = 8.0e12                           # bytes/s
BFLY_OPS = 9                                # VALU ops of one lazy Harvey butterfly
MAC_OPS = 7                                 # Montgomery product + modular add
GARNER_OPS = 14                             # two modular products, three adds or reductions


# HBM-side bytes per job of the key-switch inner kernel on this workload
# (batch 64, 8 key sets): rocprofv3 FETCH_SIZE and WRITE_SIZE summed over the
# batched launches, each scaled by that counter's reading for a 1 GiB device
# copy (FETCH_SIZE read 0.5 GiB: x2.0; WRITE_SIZE read 1 GiB: x1.0).  These
# count L2 misses, so reads served by the last-level cache count too.  Valid
# only for kernel sources with this digest; otherwise the traffic is null.
KS_INNER_TRAFFIC = {"digest": "b210ac9b93f1b31b", "fetch_per_job": 3.5944e6, "write_per_job": 1.1796e6, "K": 2}
# parameter set of the MNIST-shaped workload (--params): seven ciphertext
# primes with key-switching digits of two primes and two special primes
MNIST_PARAMS = "mnist_n16384_k2"
# the other networks' parameter sets (two-prime key-switching digits as well)
DENSE_PARAMS, HEAD_PARAMS, CIFAR_PARAMS = "mnist_dense_n16384_k2", "head_n16384_k2", "cifar_n16384_k2"
KS_INNER_SOURCES = ["keyswitch.hip", "ks_core.hpp", "ntt_core.hpp", "modarith.hpp", "lola_internal.hpp"]


def ks_inner_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KS_INNER_SOURCES:
        with open(os.path.join(ROOT, "paper_1812_10659_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def ks_shape(L, K):
    """Key-switching digits (K consecutive ciphertext primes each), target
    moduli L + K, the (target, digit) pairs that need a transform, and those
    whose digit has two primes (a Garner step each)."""
    dn = -(-L // K)
    M = L + K
    widths = [min(K, L - d * K) for d in range(dn)]
    X = dn * M - L
    G = sum(M - w for w in widths if w == 2)
    return dn, M, X, G


def ks_inner_ops(N, L, K=1):
    """Algorithmic VALU lane-ops of one key switch in the inner kernel: a
    transform of N/2 log2 N butterflies for every (target modulus, digit)
    pair whose digit does not hold the target (L^2 with one special prime)
    plus two inverse transforms per special prime, 2 dn (L+K) N
    multiply-accumulates, and a Garner step per coefficient of a two-prime
    digit's pairs."""
    dn, M, X, G = ks_shape(L, K)
    bfly = (X + 2 * K) * (N // 2) * int(math.log2(N))
    macs = 2 * dn * M * N
    return BFLY_OPS * bfly + MAC_OPS * macs + GARNER_OPS * G * N


def ks_bytes(N, L, K=1):
    """Algorithmic HBM bytes of one key switch: ciphertext in (2 L N words),
    key read once (2 dn (L+K) N words), result out (2 L N words)."""
    dn, M, _, _ = ks_shape(L, K)
    return 4 * N * (4 * L + 2 * dn * M)


def valu_probe_run(iters=4000, reps=3):
    """The library's VALU probe: eight independent chains of one 32-bit
    instruction per thread over the whole GPU, best of reps, as lane-ops/s
    and as a fraction of 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz."""
    import torch
    from paper_1812_10659_amd import lola
    props = torch.cuda.get_device_properties(0)
    out = {"metric": "VALU lane-instructions/s", "peak_lane_ops_per_s": PEAK_VALU_LANE_OPS,
           "compute_units": props.multi_processor_count, "gpu": props.name, "rates": {}}
    for op, name in enumerate(("v_mul_lo_u32", "v_mul_hi_u32", "v_add_u32")):
        lola.valu_probe(op, 10)   # warm up
        best = max(lola.valu_probe(op, iters) for _ in range(reps))
        out["rates"][name] = {"lane_ops_per_s": round(best / 1e12, 3) * 1e12,
                              "frac_of_peak": round(best / PEAK_VALU_LANE_OPS, 4)}
    return out


def inner_bytes(N, L, K=1):
    """Algorithmic HBM bytes of the inner kernel per key switch: the key, the
    limbs x and permuted limbs X' in, the accumulators U and u_P out."""
    dn, M, _, _ = ks_shape(L, K)
    return 8 * N * (dn * M + 2 * L + K)


def ks_ops(N, L, K=1):
    """Algorithmic VALU lane-ops of one whole key switch: L INTTs of the
    digit stage, the inner kernel's work, and 2L mod-down units of one NTT
    and ~10 ops a coefficient (plus a Garner step with two special primes)."""
    T = BFLY_OPS * (N // 2) * int(math.log2(N))
    return L * T + ks_inner_ops(N, L, K) + 2 * L * (T + 10 * N + (GARNER_OPS * N if K > 1 else 0))


def kernel_table(stats, steps):
    """Per timed kernel: launches, work units and the library's algorithmic
    bytes and lane-ops per launch, the average event time of a launch, and
    the fractions of the HBM and VALU peaks; the binding fraction is the
    larger (the kernel's time against max(bytes / 8 TB/s, ops / 39.3 T))."""
    out = {}
    for name, k in sorted(stats.items(), key=lambda kv: -kv[1]["ms"]):
        n = max(k["launches"], 1)
        sec = k["ms"] / 1e3
        hb = k["alg_bytes"] / sec / PEAK_HBM if sec > 0 else 0.0
        va = k["alg_ops"] / sec / PEAK_VALU_LANE_OPS if sec > 0 else 0.0
        out[name] = {"launches": k["launches"], "launches_per_step": round(k["launches"] / steps, 1),
                     "units_per_launch": round(k["units"] / n, 2),
                     "alg_bytes_per_launch": round(k["alg_bytes"] / n), "alg_ops_per_launch": round(k["alg_ops"] / n),
                     "avg_launch_ms": round(k["ms"] / n, 5), "ms_per_step": round(k["ms"] / steps, 4),
                     "hbm_frac": round(hb, 4), "valu_frac": round(va, 4),
                     "bound": "hbm" if hb >= va else "alu", "binding_frac": round(max(hb, va), 4)}
    return out


KS_KERNELS = ("ks_digits_kernel", "ks_inner_kernel", "ks_moddown_kernel",
              "ks_term_kernel", "ks_fold_kernel", "ks_term_direct_kernel", "ks_fold_moddown_kernel")


def whole_keyswitch(stats, N, L, K=1):
    """The whole key switch (digits, inner and mod-down kernels, or a small
    launch's latency-form kernels) per job over all key switches of the timed
    pass: time, algorithmic HBM GB/s and VALU fraction.  Hoisted rotations
    run other kernels and are not counted here."""
    names = [n for n in KS_KERNELS if n in stats]
    jobs = sum(stats[n]["units"] for n in ("ks_inner_kernel", "ks_term_kernel", "ks_term_direct_kernel")
               if n in stats)
    ms = sum(stats[n]["ms"] for n in names)
    if jobs == 0 or ms <= 0:
        return None
    sec = ms / 1e3
    gbps = ks_bytes(N, L, K) * jobs / sec / 1e9
    valu = ks_ops(N, L, K) * jobs / sec / PEAK_VALU_LANE_OPS
    split = {n: round(stats[n]["ms"] / jobs * 1e3, 3) for n in names}
    return {"jobs": jobs, "us_per_job": round(ms / jobs * 1e3, 3), "us_per_job_by_kernel": split,
            "gbps": round(gbps, 1), "hbm_frac": round(gbps * 1e9 / PEAK_HBM, 4),
            "ops_per_job": ks_ops(N, L, K), "valu_frac": round(valu, 4),
            "bytes_per_job": ks_bytes(N, L, K), "special_primes": K, "digits": ks_shape(L, K)[0],
            "note": "4N(4L + 2 dn (L+K)) bytes (ciphertext in, key once, result out) and the three kernels' "
                    "algorithmic lane-ops per key switch, over their summed HIP-event time"}


def main():
    global MNIST_PARAMS
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=64, help="requests per step")
    ap.add_argument("--clients", type=int, default=8, help="distinct key sets")
    ap.add_argument("--latency-runs", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-primitive run")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="mixed Poisson serving run after the timed steps (0 = skip)")
    ap.add_argument("--serve-high-rate", type=float, default=800.0,
                    help="arrival rate of a second serving run above what one-at-a-time can sustain (0 = skip)")
    ap.add_argument("--serve-saturation-rate", type=float, default=4000.0,
                    help="arrival rate of a third serving run, above what the GPU can sustain (0 = skip)")
    ap.add_argument("--no-integer-logits", action="store_true",
                    help="skip the run under seven plaintext moduli (exact integer logits by CRT)")
    ap.add_argument("--lanes", type=int, default=2, choices=(1, 2),
                    help="lanes of the batched evaluation (2: halves of the batch on two streams)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed MNIST steps and latency runs: no other network, batched, serving "
                         "or CPU section (for profiler runs whose per-kernel sums must cover that workload alone)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device-to-device once (scale for HBM counters) and exit")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default NTT and key-switch variants (no autotuning before the timed steps)")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="only run the CPU oracle on whole workloads (dense-64 query, MNIST-shaped network, "
                         "transfer head in both recipes) on all host threads and on one, and exit")
    ap.add_argument("--cpu-workloads", default="cfg0,cfg1,cfg3d,cfg3s",
                    help="with --cpu-baseline-full: which workloads (cfg0 dense-64, cfg1 MNIST-shaped, "
                         "cfg3d / cfg3s transfer head dense / stacked recipe)")
    ap.add_argument("--cpu-threads", default="all,1",
                    help="with --cpu-baseline-full: thread counts ('all' = every host thread)")
    ap.add_argument("--params", default=MNIST_PARAMS, choices=("mnist_n16384", "mnist_n16384_k2"),
                    help="parameter set of the MNIST-shaped workload: one special prime and a key-switching "
                         "digit per ciphertext prime, or two special primes and digits of two primes")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only measure the 32-bit VALU issue rates (mul_lo, mul_hi, add) against the "
                         "CU x SIMD x lane x clock peak and exit")
    args = ap.parse_args()
    if args.valu_probe:
        print(json.dumps(valu_probe_run()), flush=True)
        return
    if args.cpu_baseline_full:
        print(json.dumps(cpu_baseline_full(args.cpu_workloads.split(","), args.cpu_threads.split(","))), flush=True)
        return
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes": src.numel() * 4}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a deployment would shard requests across GPUs, one process per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1812_10659_amd import lola, networks
    from paper_1812_10659_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    serving_out = {}
    if args.serve_requests > 0 and not args.headline_only:
        # Serving first, in a process that has created no other streams yet:
        # the host drives every scheduling round, and each model runs on two
        # streams of its own, which measured 20% slower at saturation once
        # the headline's streams existed (2745/s against 3345-3700/s).
        # Poisson arrivals: 70% N=16384 MNIST-shaped, 30% N=4096 dense-64,
        # 8 resident key sets per ring size, continuous batching vs one at a time.
        from paper_1812_10659_amd import serving
        serving_out["serving"] = serving.run_serving(n_req=args.serve_requests, mnist_params=args.params)
        if args.serve_high_rate > 0:
            serving_out["serving_high_load"] = serving.run_serving(n_req=args.serve_requests,
                                                                   rate=args.serve_high_rate,
                                                                   mnist_params=args.params)
        if args.serve_saturation_rate > 0:
            serving_out["serving_saturation"] = serving.run_serving(n_req=args.serve_requests,
                                                                    rate=args.serve_saturation_rate,
                                                                    mnist_params=args.params)
        torch.cuda.empty_cache()
    MNIST_PARAMS = args.params
    p = wl.PARAMS[MNIST_PARAMS]
    N, L, K = p.N, p.L, len(p.special)
    w = wl.mnist_weights()
    ctx = lola.Context(p)
    plan = lola.Plan(p, networks.mnist_layers(w))
    plan.load(ctx)
    plan.set_lanes(args.lanes)
    tuned = None
    if not args.no_autotune:
        # radix splits, LDS placements and tiles of the batched NTT and of the
        # three key-switch stages, timed on the device (each variant checked
        # word for word against the default first) and cached per (N, L)
        from paper_1812_10659_amd import batched
        ntt_c, ks_c = batched.autotune_ntt(ctx, N, L), batched.autotune_ks(ctx, N, L)
        tuned = {"ntt": {"chosen": dict(zip(("split", "limbs_per_wg"), ctx.ntt_variants()[ctx.ntt_variant()])),
                         "trials_ms": ntt_c.get("ntt_trials_ms")},
                 "keyswitch": {"chosen": {lola.KS_STAGES[st]: dict(zip(("split", "padded"),
                                                                       ctx.ks_variants(st)[ctx.ks_variant(st)]))
                                          for st in range(3)},
                               "trials_ms": ks_c.get("ks_trials_ms"), "trial_jobs": ks_c.get("ks_trial_jobs")}}
    from paper_1812_10659_amd import requests as rq
    B, C = args.batch, max(1, min(args.clients, args.batch))
    reqs, keys, images = rq.mnist_batch(ctx, plan, B, C)
    torch.cuda.synchronize()

    # warmup (also binds the batch: descriptors uploaded once)
    for _ in range(args.warmup):
        plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    # value: the batch as the library runs it (two lanes on two streams)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the same steps replayed through a HIP graph (captured once, with the
    # same two lanes) on a stream of its own
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        plan.evaluate(ctx, reqs, graph=True, stream=gs)   # capture
        gs.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            plan.evaluate(ctx, reqs, graph=True, stream=gs)
        gs.synchronize()
        elapsed_graph = time.perf_counter() - tg
    # roofline: the same steps with the key-switch inner kernel timed by HIP
    # events on its launch stream; kernel timing runs the batch as one lane,
    # so every launch is timed alone
    lola.timing_enable(ctx, True)
    plan.evaluate(ctx, reqs)                     # binds the one-lane program
    torch.cuda.synchronize()
    lola.kernel_timing(ctx)                      # drain
    t1 = time.perf_counter()
    for _ in range(args.steps):
        plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    elapsed_one_lane = time.perf_counter() - t1
    lola.timing_enable(ctx, False)
    kstats = lola.kernel_stats(ctx)

    # every request of the timed batch decrypts to the plain network's logits
    for r in range(B):
        got = rq.decrypted_outputs(ctx, plan, keys[r % C]["sk"], reqs[r])
        exp = _plain_logits_mod_t(images[r], w, p.t)
        assert [int(v) for v in got] == [int(v) for v in exp], f"request {r}: decrypted logits differ"

    # single-request latency (unbatched path, eager)
    lat = []
    one = [reqs[0]]
    plan.evaluate(ctx, one)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    for _ in range(args.latency_runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.evaluate(ctx, one)
        e1.record(s)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    lat = np.array(lat)
    # the same, replayed through a HIP graph
    lat_g = []
    with torch.cuda.stream(gs):
        plan.evaluate(ctx, one, graph=True, stream=gs)   # capture
        gs.synchronize()
        for _ in range(args.latency_runs):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(gs)
            plan.evaluate(ctx, one, graph=True, stream=gs)
            e1.record(gs)
            e1.synchronize()
            lat_g.append(e0.elapsed_time(e1))
    lat_g = np.array(lat_g)
    # client-inclusive latency of one request: pack the image's slots on the
    # host, encode them (one host to device copy) and encrypt them into the
    # request's resident input block, evaluate, then decrypt and decode the
    # output block and bring the logits back to the host (one copy)
    imap_np, omap_np = plan.input_map(), plan.output_map()
    k0 = keys[0]
    cin = ctx.empty(len(reqs[0]["inputs"]), 2, L, N)
    cout = ctx.empty(plan.info["n_outputs"], 2, L, N)
    creq = [dict(rlk=k0["rlk"], gks=k0["gks"], inputs=list(cin), outputs=list(cout))]

    def client_run():
        msgs = networks.pack_inputs(imap_np, networks.mnist_input_values(images[0]))
        ctx.encrypt_batch(k0["pk"], ctx.encode_batch(msgs), wl.enc_seed(1), 0, out=cin)
        plan.evaluate(ctx, creq)
        slots = ctx.decode_batch(ctx.decrypt_batch(k0["sk"], cout)).cpu().numpy()
        return networks.unpack_outputs(omap_np, slots)

    client_run()   # binds the request
    lat_c = []
    for _ in range(args.latency_runs):
        tc = time.perf_counter()
        logits = client_run()
        lat_c.append((time.perf_counter() - tc) * 1e3)
    lat_c = np.array(lat_c)
    exp0 = _plain_logits_mod_t(images[0], w, p.t)
    assert [int(v) for v in logits] == [int(v) for v in exp0], "client-inclusive run: decrypted logits differ"

    # NTT throughput: batched forward transforms of 7*512 limbs
    nl = 7 * 512
    x = torch.randint(0, 1 << 29, (nl, N), dtype=torch.int32, device="cuda")
    idx = np.arange(nl, dtype=np.uint32) % L   # built once, as a caller would
    ctx.ntt_limbs(x, idx)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 5
    for _ in range(reps):
        ctx.ntt_limbs(x, idx)
    e1.record()
    e1.synchronize()
    ntt_s = e0.elapsed_time(e1) / 1e3 / reps
    ntt_gbps = nl * 8 * N / ntt_s / 1e9

    ms_per_step = elapsed / args.steps * 1e3
    value = B * args.steps / elapsed
    kernels = kernel_table(kstats, args.steps)
    inner = kstats.get("ks_inner_kernel", dict(ms=0.0, launches=0, units=0, alg_ops=0.0, alg_bytes=0.0))
    ks_jobs, ks_launches, ks_ms = inner["units"], inner["launches"], inner["ms"]
    ops_per_job = ks_inner_ops(N, L, K)
    ks_avg_ms = ks_ms / max(ks_launches, 1)
    jobs_per_launch = ks_jobs / max(ks_launches, 1)
    achieved = ops_per_job * ks_jobs / (ks_ms / 1e3) if ks_ms > 0 else 0.0
    whole_ks = whole_keyswitch(kstats, N, L, K)
    traffic = None
    if ks_inner_digest() == KS_INNER_TRAFFIC["digest"] and (B, C) == (64, 8) and K == KS_INNER_TRAFFIC["K"]:
        tb = (KS_INNER_TRAFFIC["fetch_per_job"] + KS_INNER_TRAFFIC["write_per_job"]) * jobs_per_launch
        traffic = {"bytes_per_launch": round(tb), "algorithmic_bytes_per_launch": round(inner_bytes(N, L, K) * jobs_per_launch),
                   "gbps": round(tb / (ks_avg_ms / 1e3) / 1e9, 1)}

    out = {
        "metric": "encrypted inferences/s (N=16384 MNIST-shaped LoLa network)",
        "value": round(value, 2),
        "unit": "inferences/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 (RNS residues mod 30-bit primes)",
        "data": "synthetic (seeded uniform 28x28 images, seeded int8 weights)",
        "config": {"workload": "MNIST-shaped: conv5x5s2x5 -> sq -> fc845x100 -> sq -> fc100x10, "
                               "BFV N=16384 L=7 t=1146881",
                   "params": p.name, "special_primes": K, "keyswitch_digits": ks_shape(L, K)[0],
                   "plan": {"recipe": RECIPE_NAMES.get(plan.info["recipe"], str(plan.info["recipe"])),
                            "rotations": plan.info["n_rotations"], "mul_plain": plan.info["n_mul_plain"],
                            "mul_scalar": plan.info["n_mul_scalar"], "squares": plan.info["n_square"],
                            "output_messages": plan.info["n_outputs"],
                            "predicted_latency_ms": round(plan.info["predicted_latency_us"] / 1e3, 3)},
                   "batch_requests": B, "client_key_sets": C, "lanes": args.lanes, "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "single_request_inferences_per_s": round(1e3 / float(np.median(lat)), 2),
                       "graph_replay_p50": round(float(np.percentile(lat_g, 50)), 3),
                       "graph_replay_p99": round(float(np.percentile(lat_g, 99)), 3),
                       "client_inclusive_p50": round(float(np.percentile(lat_c, 50)), 3),
                       "client_inclusive_p99": round(float(np.percentile(lat_c, 99)), 3),
                       "client_inclusive_note": "host packing, batched encode and encrypt of the input "
                                                "messages, evaluate, batched decrypt and decode, logits back "
                                                "on the host"},
        "graph_replay": {"ms_per_step": round(elapsed_graph / args.steps * 1e3, 3),
                         "inferences_per_s": round(B * args.steps / elapsed_graph, 2),
                         "note": "the timed steps replayed from one captured HIP graph"},
        "roofline": {"bound": "alu", "kernel": "ks_inner_kernel<14>",
                     "achieved": round(achieved / 1e12, 3), "peak": round(PEAK_VALU_LANE_OPS / 1e12, 1),
                     "unit": "T VALU lane-ops/s", "frac": round(achieved / PEAK_VALU_LANE_OPS, 4),
                     "traffic": traffic and traffic["bytes_per_launch"], "traffic_detail": traffic,
                     "avg_launch_ms": round(ks_avg_ms, 4),
                     "jobs_per_launch": round(jobs_per_launch, 1), "ops_per_job": ops_per_job,
                     "note": "ops_per_job is the inner product's algorithmic lane-op count for the context's "
                             "key-switching shape (digits of two primes: fewer transforms and key products than "
                             "one prime per digit, whose figures are under other_keyswitch_shape)",
                     "pass": f"{args.steps} steps of the same batch and plan after the timed ones, run as one "
                             f"lane so that each launch is timed alone "
                             f"({B * args.steps / elapsed_one_lane:.1f} inferences/s in that pass)"},
        "hbm": {"ntt_gbps": round(ntt_gbps, 1), "ntt_frac": round(ntt_gbps * 1e9 / PEAK_HBM, 4),
                "keyswitch_gbps": whole_ks and whole_ks["gbps"],
                "keyswitch_frac": whole_ks and whole_ks["hbm_frac"],
                "note": "algorithmic bytes: NTT 8N per limb; key switch 4N(4L + 2 dn (L+K)) per job over the "
                        "summed time of its three kernels (digits, inner, mod-down) in the timed pass"},
        "keyswitch": whole_ks,
        "kernels": kernels,
        "autotune": tuned,
        "context": {"paper_latency_s": 2.2, "paper_hw": "8 vCPU Azure B8ms, SEAL 2.3.1"},
    }
    headline_recipe = plan.info["recipe"]
    if args.headline_only:
        print(json.dumps(out), flush=True)
        return
    if serving_out:
        out.update(serving_out)
    out["latency_plans"] = latency_plans_run(ctx, w, images[0], args.latency_runs)
    out["latency_ms"]["latency_plan_p50"] = out["latency_plans"]["mnist"]["latency_plan"]["p50_ms"]
    out["latency_ms"]["latency_plan_p99"] = out["latency_plans"]["mnist"]["latency_plan"]["p99_ms"]
    out["paper_layout"] = paper_layout_run(ctx, w, images, B, C, args.latency_runs)
    other = "mnist_n16384" if args.params != "mnist_n16384" else "mnist_n16384_k2"
    out["other_keyswitch_shape"] = keyswitch_shape_run(other, w, B, C, args.steps, args.warmup, args.lanes,
                                                       not args.no_autotune, args.latency_runs)
    out["mnist_small"] = small_network_run(ctx, B, C, args.latency_runs)
    out["mnist_dense_input"] = dense_input_run(B, C, args.latency_runs)
    out["cifar_shaped"] = cifar_run()
    out["head_recipes"] = head_recipes_run()
    if not args.no_integer_logits:
        del reqs, keys
        torch.cuda.empty_cache()
        out["integer_logits"] = integer_logits_run(w, B, C)
        reqs, keys = None, None
        torch.cuda.empty_cache()
    if not args.no_batched:
        # batched primitives: 512 ciphertexts, N=16384, L=8, uneven rotation chains
        from paper_1812_10659_amd import batched
        b2 = batched.run_batched()
        b2.pop("_tensors")
        out["batched_primitives"] = b2
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, w, ORACLE_RECIPE[headline_recipe])
    print(json.dumps(out), flush=True)


ORACLE_RECIPE = {4: "full", 5: "shared"}
RECIPE_NAMES = {1: "dense vector - row major", 2: "stacked vector - row major", 3: "fixed",
                4: "full reduction (the paper's layout)", 5: "shared reduction"}


def _one_request_latency(ctx, plan, req, runs):
    """p50 and p99 (ms) of one request evaluated alone, HIP events around
    each call on the current stream."""
    import numpy as np
    import torch
    one = [req]
    plan.evaluate(ctx, one)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    lat = []
    for _ in range(runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.evaluate(ctx, one)
        e1.record(s)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def _latency_plan_case(ctx, p, layers, values, expected, runs, key_seed):
    """One network under the plan compiled for the latency objective and under
    the default (throughput) plan, each timed on one request alone; the
    latency plan's outputs checked against the plain network mod t."""
    import numpy as np

    from paper_1812_10659_amd import lola
    from paper_1812_10659_amd import requests as rq
    res = {}
    for tag, obj in (("throughput_plan", lola.OBJECTIVE_THROUGHPUT), ("latency_plan", lola.OBJECTIVE_LATENCY)):
        plan = lola.Plan(p, layers, objective=obj)
        plan.load(ctx)
        key = rq.client_keys(ctx, plan, 1, key_seed)[0]
        # a plan packing several queries per message gets the same query in each
        req = rq.encrypted_request(ctx, plan, key, np.tile(np.asarray(values), plan.info["queries"]), key_seed + 1)
        p50, p99 = _one_request_latency(ctx, plan, req, runs)
        info = plan.info
        res[tag] = {"recipe": RECIPE_NAMES.get(info["recipe"], str(info["recipe"])),
                    "sums": {1: "sequential", 2: "hoisted"}.get(info["sums"], str(info["sums"])),
                    "rotations": info["n_rotations"], "levels": info["n_waves"], "galois_keys": info["n_galois"],
                    "predicted_latency_ms": round(info["predicted_latency_us"] / 1e3, 3),
                    "p50_ms": round(p50, 3), "p99_ms": round(p99, 3)}
        if obj == lola.OBJECTIVE_LATENCY:
            got = rq.decrypted_outputs(ctx, plan, key["sk"], req)
            n = len(expected)
            assert [int(v) for v in got[:n]] == [int(v) % p.t for v in expected], "latency plan: outputs differ"
            res[tag]["checked"] = 1
        plan.close()
    return res


def latency_plans_run(ctx, w, img, latency_runs):
    """Single-request latency of each network under the plan compiled for the
    latency objective (the compiler prices both forms of the sums, sequential
    and hoisted, with every candidate recipe and keeps the lowest predicted
    latency) beside the default throughput plan, both timed here the same
    way; every latency plan's outputs checked against the plain network."""
    import numpy as np

    from paper_1812_10659_amd import lola, networks
    from paper_1812_10659_amd import workloads as wl
    out = {}
    pm = wl.PARAMS[MNIST_PARAMS]
    mv = networks.mnist_input_values(img)
    out["mnist"] = _latency_plan_case(ctx, pm, networks.mnist_layers(w), mv, _plain_logits_mod_t(img, w, pm.t),
                                      latency_runs, wl.key_seed(1) + 101)
    ws = wl.mnist_small_weights()
    out["mnist_small"] = _latency_plan_case(ctx, pm, networks.mnist_small_layers(ws), mv,
                                            _plain_small_logits(img, ws), latency_runs, wl.key_seed(1) + 103)
    pd = wl.PARAMS[DENSE_PARAMS]
    out["mnist_dense_input"] = _latency_plan_case(lola.Context(pd), pd, networks.mnist_dense_layers(w), mv,
                                                  _plain_logits_mod_t(img, w, pd.t), latency_runs,
                                                  wl.key_seed(1) + 105)
    ph, wh = wl.PARAMS[HEAD_PARAMS], wl.head_weights()
    f = wl.head_features(1)[0]
    out["head"] = _latency_plan_case(lola.Context(ph), ph, networks.head_layers(wh), f, _head_plain(f, wh),
                                     latency_runs, wl.key_seed(3) + 107)
    p0 = wl.PARAMS["n4096_3q"]
    x, W = wl.dense64_inputs()
    y = W.astype(object).dot(np.asarray(x).astype(object))
    out["dense64"] = _latency_plan_case(lola.Context(p0), p0, networks.dense64_layers(W), x, list(y * y),
                                        latency_runs, wl.key_seed(0) + 109)
    return out


def paper_layout_run(ctx, w, images, B, C, latency_runs, steps=5):
    """The same network and batch compiled with the layout the paper describes
    (every stacked round summed over its block, one output message per class:
    154 rotations): batch throughput and one-request latency, two requests
    checked against the plaintext network mod t."""
    import numpy as np
    import torch
    from paper_1812_10659_amd import lola, networks
    from paper_1812_10659_amd import workloads as wl
    p = wl.PARAMS[MNIST_PARAMS]
    plan = lola.Plan(p, networks.mnist_layers(w), recipe=lola.RECIPE_FULL_REDUCTION)
    plan.load(ctx)
    keys = []
    for c in range(C):
        ks = wl.key_seed(1) + 7919 * c
        sk = ctx.keygen_secret(ks)
        keys.append(dict(sk=sk, pk=ctx.keygen_public(ks, sk), rlk=ctx.keygen_switch(ks, sk, 0),
                         gks=[ctx.keygen_switch(ks, sk, g) for g in plan.galois()]))
    imap, reqs = plan.input_map(), []
    for r in range(B):
        k = keys[r % C]
        msgs = networks.pack_inputs(imap, networks.mnist_input_values(images[r]))
        reqs.append(dict(rlk=k["rlk"], gks=k["gks"],
                         inputs=[ctx.encrypt(k["pk"], ctx.encode(m), wl.enc_seed(1) + r, i) for i, m in enumerate(msgs)],
                         outputs=[ctx.empty_ct() for _ in range(plan.info["n_outputs"])]))
    plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    for r in (0, B - 1):
        slots = np.stack([ctx.decode(ctx.decrypt(keys[r % C]["sk"], o)) for o in reqs[r]["outputs"]])
        got = networks.unpack_outputs(plan.output_map(), slots)
        exp = _plain_logits_mod_t(images[r], w, p.t)
        assert [int(v) for v in got] == [int(v) for v in exp], f"paper layout request {r} differs"
    lat = []
    one = [reqs[0]]
    s = torch.cuda.current_stream()
    for _ in range(latency_runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.evaluate(ctx, one)
        e1.record(s)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    out = {"recipe": RECIPE_NAMES[plan.info["recipe"]], "rotations": plan.info["n_rotations"],
           "output_messages": plan.info["n_outputs"], "batch_requests": B,
           "predicted_latency_ms": round(plan.info["predicted_latency_us"] / 1e3, 3),
           "inferences_per_s": round(B / dt, 1), "ms_per_batch": round(dt * 1e3, 3),
           "latency_p50_ms": round(float(np.percentile(lat, 50)), 3),
           "latency_p99_ms": round(float(np.percentile(lat, 99)), 3), "checked": 2}
    del reqs, keys, plan
    torch.cuda.empty_cache()
    return out


def small_network_run(ctx, B, C, latency_runs, steps=5):
    """The small variant (convolution, square, dense 845 -> 10; 18 rotations,
    one square) on the same context: batch throughput and one-request
    latency; two requests checked against the plaintext network mod t."""
    import numpy as np
    import torch
    from paper_1812_10659_amd import lola, networks
    from paper_1812_10659_amd import workloads as wl
    w = wl.mnist_small_weights()
    p = wl.PARAMS[MNIST_PARAMS]
    plan = lola.Plan(p, networks.mnist_small_layers(w))
    plan.load(ctx)
    keys = []
    for c in range(C):
        ks = wl.key_seed(1) + 7919 * c + 1
        sk = ctx.keygen_secret(ks)
        keys.append(dict(sk=sk, pk=ctx.keygen_public(ks, sk), rlk=ctx.keygen_switch(ks, sk, 0),
                         gks=[ctx.keygen_switch(ks, sk, g) for g in plan.galois()]))
    imap, imgs, reqs = plan.input_map(), [], []
    for r in range(B):
        img = wl.mnist_image(index=r)
        imgs.append(img)
        k = keys[r % C]
        msgs = networks.pack_inputs(imap, networks.mnist_input_values(img))
        reqs.append(dict(rlk=k["rlk"], gks=k["gks"],
                         inputs=[ctx.encrypt(k["pk"], ctx.encode(m), wl.enc_seed(1) + 100 + r, i) for i, m in enumerate(msgs)],
                         outputs=[ctx.empty_ct()]))
    plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    for r in (0, B - 1):
        got = networks.unpack_outputs(plan.output_map(), np.stack([ctx.decode(ctx.decrypt(keys[r % C]["sk"], reqs[r]["outputs"][0]))]))
        exp = [(int(v) % p.t) for v in _plain_small_logits(imgs[r], w)]
        assert [int(v) for v in got] == exp, f"small network request {r} differs"
    lat = []
    one = [reqs[0]]
    s = torch.cuda.current_stream()
    for _ in range(latency_runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.evaluate(ctx, one)
        e1.record(s)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    return {"layers": "conv5x5s2x5 -> sq -> fc845x10", "rotations": plan.info["n_rotations"],
            "batch_requests": B, "inferences_per_s": round(B / dt, 1), "ms_per_batch": round(dt * 1e3, 3),
            "latency_p50_ms": round(float(np.percentile(lat, 50)), 3), "paper_latency_s": 0.29, "checked": 2}


def dense_input_run(B, C, latency_runs, steps=3):
    """LoLa-Dense: the same network with the image sent as one dense message
    (25 masks and 24 more rotations build the convolution messages; 256
    rotations, eight data primes).  Batch throughput and one-request latency;
    two requests checked against the plaintext network mod t."""
    import numpy as np
    import torch
    from paper_1812_10659_amd import lola, networks
    from paper_1812_10659_amd import workloads as wl
    p = wl.PARAMS[DENSE_PARAMS]
    w = wl.mnist_weights()
    ctx = lola.Context(p)
    plan = lola.Plan(p, networks.mnist_dense_layers(w))
    plan.load(ctx)
    keys = []
    for c in range(C):
        ks = wl.key_seed(1) + 7919 * c + 2
        sk = ctx.keygen_secret(ks)
        keys.append(dict(sk=sk, pk=ctx.keygen_public(ks, sk), rlk=ctx.keygen_switch(ks, sk, 0),
                         gks=[ctx.keygen_switch(ks, sk, g) for g in plan.galois()]))
    imap, imgs, reqs = plan.input_map(), [], []
    for r in range(B):
        img = wl.mnist_image(index=r)
        imgs.append(img)
        k = keys[r % C]
        msgs = networks.pack_inputs(imap, networks.mnist_input_values(img))
        reqs.append(dict(rlk=k["rlk"], gks=k["gks"],
                         inputs=[ctx.encrypt(k["pk"], ctx.encode(m), wl.enc_seed(1) + 200 + r, i) for i, m in enumerate(msgs)],
                         outputs=[ctx.empty_ct() for _ in range(plan.info["n_outputs"])]))
    plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    for r in (0, B - 1):
        slots = np.stack([ctx.decode(ctx.decrypt(keys[r % C]["sk"], o)) for o in reqs[r]["outputs"]])
        got = networks.unpack_outputs(plan.output_map(), slots)
        assert [int(v) for v in got] == [int(v) for v in _plain_logits_mod_t(imgs[r], w, p.t)], f"dense-input request {r} differs"
    lat = []
    s = torch.cuda.current_stream()
    for _ in range(latency_runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        plan.evaluate(ctx, reqs[:1])
        e1.record(s)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    return {"input": "one dense message (padded 29x29 image)", "data_primes": p.L,
            "rotations": plan.info["n_rotations"], "batch_requests": B,
            "inferences_per_s": round(B / dt, 1), "ms_per_batch": round(dt * 1e3, 3),
            "latency_p50_ms": round(float(np.percentile(lat, 50)), 3), "paper_latency_s": 7.2, "checked": 2}


def head_recipes_run(n_queries=64, steps=3):
    """The transfer-learning head (4096 -> 256 -> square -> 10) under both
    recipes the compiler prices: dense vector - row major with 4 queries per
    message, and stacked vector - row major with one.  Measured time per query
    for a batch of n_queries and for one query alone, beside the cost model's
    prediction; both checked against the plaintext head mod t."""
    import numpy as np
    import torch
    from paper_1812_10659_amd import lola, networks
    from paper_1812_10659_amd import workloads as wl
    p = wl.PARAMS[HEAD_PARAMS]
    w = wl.head_weights()
    feats = wl.head_features(n_queries)
    exp = [[int(v) % p.t for v in _head_plain(feats[q], w)] for q in range(n_queries)]
    ctx = lola.Context(p)
    res = {}
    for name, rec in (("dense_row_major", lola.RECIPE_DENSE_ROW_MAJOR), ("stacked_row_major", lola.RECIPE_STACKED_ROW_MAJOR)):
        plan = lola.Plan(p, networks.head_layers(w), recipe=rec)
        plan.load(ctx)
        Q = plan.info["queries"]
        ks = wl.key_seed(3) + rec
        sk = ctx.keygen_secret(ks)
        pk = ctx.keygen_public(ks, sk)
        rlk, gks = ctx.keygen_switch(ks, sk, 0), [ctx.keygen_switch(ks, sk, g) for g in plan.galois()]
        reqs = []
        for m in range(n_queries // Q):
            vals = feats[m * Q:(m + 1) * Q].reshape(-1)
            msgs = networks.pack_inputs(plan.input_map(), vals)
            reqs.append(dict(rlk=rlk, gks=gks, inputs=[ctx.encrypt(pk, ctx.encode(x), 77 + m, i) for i, x in enumerate(msgs)],
                             outputs=[ctx.empty_ct() for _ in range(plan.info["n_outputs"])]))
        plan.evaluate(ctx, reqs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.evaluate(ctx, reqs)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        t1 = time.perf_counter()
        plan.evaluate(ctx, reqs[:1])
        torch.cuda.synchronize()
        one = time.perf_counter() - t1
        for m in (0, len(reqs) - 1):
            slots = np.stack([ctx.decode(ctx.decrypt(sk, o)) for o in reqs[m]["outputs"]])
            got = networks.unpack_outputs(plan.output_map(), slots).reshape(Q, -1)
            for q in range(Q):
                assert [int(v) for v in got[q]] == exp[m * Q + q], f"head {name}: query {m * Q + q} differs"
        res[name] = {"queries_per_message": Q, "rotations_per_message": plan.info["n_rotations"],
                     "batch_ms_per_query": round(dt * 1e3 / n_queries, 4),
                     "one_message_ms": round(one * 1e3, 3),
                     "predicted_us_per_message": round(float(plan.info["predicted_us"]), 1),
                     "predicted_latency_ms": round(float(plan.info["predicted_latency_us"]) / 1e3, 3)}
    res["chosen"] = {"throughput": lola.Plan(p, networks.head_layers(w), objective=lola.OBJECTIVE_THROUGHPUT).info["recipe"],
                     "latency": lola.Plan(p, networks.head_layers(w), objective=lola.OBJECTIVE_LATENCY).info["recipe"],
                     "codes": {"1": "dense_row_major", "2": "stacked_row_major"}}
    res["batch_queries"] = n_queries
    return res


def _head_plain(f, w):
    h = w.w1.astype(object).dot(f.astype(object)) + w.b1.astype(object)
    return w.w2.astype(object).dot(h * h) + w.b2.astype(object)


def cifar_run(runs=3):
    """The collapsed CIFAR network of Sec. 4.4 (8x8x3 convolution, 83 maps;
    square; 6x6x83 convolution, 163 maps, as dense vector - row major; square;
    dense 4075 -> 10): 57251 rotations for one image.  Latency of one
    encrypted image (eight data primes); decrypted logits checked against the
    plaintext network mod t."""
    import numpy as np
    import torch
    from paper_1812_10659_amd import lola, networks
    from paper_1812_10659_amd import workloads as wl
    p = wl.PARAMS[CIFAR_PARAMS]
    w = wl.cifar_weights()
    img = wl.cifar_image(index=0)
    t0 = time.perf_counter()
    plan = lola.Plan(p, networks.cifar_layers(w))
    compile_s = time.perf_counter() - t0
    ctx = lola.Context(p)
    plan.load(ctx)
    ks = wl.key_seed(5)
    sk = ctx.keygen_secret(ks)
    pk = ctx.keygen_public(ks, sk)
    msgs = networks.pack_inputs(plan.input_map(), networks.cifar_input_values(img))
    req = dict(rlk=ctx.keygen_switch(ks, sk, 0), gks=[ctx.keygen_switch(ks, sk, g) for g in plan.galois()],
               inputs=[ctx.encrypt(pk, ctx.encode(m), wl.enc_seed(5), i) for i, m in enumerate(msgs)],
               outputs=[ctx.empty_ct() for _ in range(plan.info["n_outputs"])])
    plan.evaluate(ctx, [req])
    torch.cuda.synchronize()
    lat = []
    for _ in range(runs):
        t1 = time.perf_counter()
        plan.evaluate(ctx, [req])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
    slots = np.stack([ctx.decode(ctx.decrypt(sk, o)) for o in req["outputs"]])
    got = networks.unpack_outputs(plan.output_map(), slots)
    exp = _cifar_plain_mod_t(img, w, p.t)
    assert [int(v) for v in got] == exp, "CIFAR-shaped logits differ from the network"
    info = plan.info
    return {"layers": "conv8x8x3s2x83 -> sq -> conv6x6x83s2x163 -> sq -> fc4075x10", "data_primes": p.L,
            "rotations": info["n_rotations"], "mul_plain": info["n_mul_plain"], "squares": info["n_square"],
            "latency_s": round(float(np.median(lat)), 4), "rotations_per_s": round(info["n_rotations"] / float(np.median(lat)), 1),
            "compile_s": round(compile_s, 2), "paper_latency_s": 730, "checked": 1}


def _cifar_plain_mod_t(img, w, t):
    """The CIFAR-shaped network on plaintext integers mod t (image padded by
    one pixel on every side)."""
    import numpy as np
    x = np.zeros((3, 34, 34), dtype=np.int64)
    x[:, 1:33, 1:33] = img

    def conv(x, wt, b):
        M, C, k, _ = wt.shape
        n = (x.shape[1] - k) // 2 + 1
        out = np.zeros((M, n, n), dtype=np.int64)
        for y in range(n):
            for xx in range(n):
                win = x[:, 2 * y:2 * y + k, 2 * xx:2 * xx + k].reshape(-1)
                out[:, y, xx] = (wt.reshape(M, -1) % t).dot(win % t) % t
        return (out + b[:, None, None]) % t

    a1 = conv(x, w.conv1_w, w.conv1_b)
    a1 = a1 * a1 % t
    a2 = conv(a1, w.conv2_w, w.conv2_b)
    a2 = (a2 * a2 % t).reshape(-1)
    return [int(v) for v in ((w.w3 % t).dot(a2) + w.b3) % t]


def _plain_small_logits(img, w):
    """The small network on plaintext Python integers."""
    import numpy as np
    pad = np.zeros((29, 29), dtype=object)
    pad[:28, :28] = img
    a1 = []
    for m in range(5):
        for y in range(13):
            for x in range(13):
                v = int((pad[2 * y:2 * y + 5, 2 * x:2 * x + 5] * w.conv_w[m].astype(object)).sum()) + int(w.conv_b[m])
                a1.append(v * v)
    return [sum(int(a) * int(b) for a, b in zip(row, a1)) + int(bb) for row, bb in zip(w.w, w.b)]


def integer_logits_run(w, B, C, steps=3):
    """The same network and batch under the seven plaintext moduli of the CRT
    set: one encrypted evaluation per modulus, exact integer logits from the
    device combination; two requests checked against the integer network."""
    import torch
    from paper_1812_10659_amd import crt, networks
    from paper_1812_10659_amd import workloads as wl
    net = crt.CrtNetwork(wl.crt_params(), networks.mnist_layers(w))
    keys = [net.keygen(wl.key_seed(1) + 7919 * c + 3) for c in range(C)]
    imgs = [wl.mnist_image(index=r) for r in range(B)]
    reqs = [net.request(keys[r % C], networks.mnist_input_values(imgs[r]), wl.enc_seed(1) + r) for r in range(B)]
    net.evaluate(reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.evaluate(reqs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    t1 = time.perf_counter()
    got = [net.integers(keys[r % C], reqs[r]) for r in (0, B - 1)]
    torch.cuda.synchronize()
    dec_ms = (time.perf_counter() - t1) / 2 * 1e3
    for r, g in zip((0, B - 1), got):
        assert g == _plain_logits_exact(imgs[r], w), f"request {r}: integer logits differ from the network"
    mx = max(abs(v) for g in got for v in g)
    return {"moduli": list(net.moduli), "requests": B, "ms_per_batch": round(dt * 1e3, 3),
            "inferences_per_s": round(B / dt, 2), "decrypt_and_combine_ms_per_request": round(dec_ms, 3),
            "max_abs_logit_bits": round(math.log2(mx), 1) if mx else 0.0,
            "product_of_moduli_bits": round(math.log2(math.prod(net.moduli)), 1), "checked": 2}


def _plain_logits_exact(img, w):
    """The network on plaintext Python integers (no reduction)."""
    import numpy as np
    pad = np.zeros((29, 29), dtype=object)
    pad[:28, :28] = img
    wc = w.conv_w.astype(object)
    a1 = []
    for m in range(5):
        for y in range(13):
            for x in range(13):
                v = int((pad[2 * y:2 * y + 5, 2 * x:2 * x + 5] * wc[m]).sum()) + int(w.conv_b[m])
                a1.append(v * v)
    h = [sum(int(a) * int(b) for a, b in zip(row, a1)) + int(bb) for row, bb in zip(w.w1, w.b1)]
    a2 = [v * v for v in h]
    return [sum(int(a) * int(b) for a, b in zip(row, a2)) + int(bb) for row, bb in zip(w.w2, w.b2)]


def keyswitch_shape_run(pname, w, B, C, steps, warmup, lanes, tune, latency_runs):
    """The headline batch under the other key-switching shape (one prime per
    digit with one special prime, or digits of two primes with two): the same
    network, batch, lanes and autotuning, timed the same way; the one-lane
    kernel-timing pass gives the whole key switch per job; every request
    decrypts to the plain network's logits."""
    import numpy as np
    import torch

    from paper_1812_10659_amd import lola, networks
    from paper_1812_10659_amd import requests as rq
    from paper_1812_10659_amd import workloads as wl
    p = wl.PARAMS[pname]
    ctx = lola.Context(p)
    plan = lola.Plan(p, networks.mnist_layers(w))
    plan.load(ctx)
    plan.set_lanes(lanes)
    if tune:
        from paper_1812_10659_amd import batched
        batched.autotune_ntt(ctx, p.N, p.L)
        batched.autotune_ks(ctx, p.N, p.L)
    reqs, keys, images = rq.mnist_batch(ctx, plan, B, C)
    for _ in range(warmup):
        plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lola.timing_enable(ctx, True)
    plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    lola.kernel_timing(ctx)
    for _ in range(steps):
        plan.evaluate(ctx, reqs)
    torch.cuda.synchronize()
    lola.timing_enable(ctx, False)
    kst = lola.kernel_stats(ctx)
    whole = whole_keyswitch(kst, p.N, p.L, len(p.special))
    inner = kst.get("ks_inner_kernel")
    inner_frac = (ks_inner_ops(p.N, p.L, len(p.special)) * inner["units"] / (inner["ms"] / 1e3) / PEAK_VALU_LANE_OPS
                  if inner and inner["ms"] > 0 else None)
    for r in range(B):
        got = rq.decrypted_outputs(ctx, plan, keys[r % C]["sk"], reqs[r])
        assert [int(v) for v in got] == [int(v) for v in _plain_logits_mod_t(images[r], w, p.t)], f"request {r}"
    one = [reqs[0]]
    plan.evaluate(ctx, one)
    torch.cuda.synchronize()
    lat = []
    for _ in range(latency_runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.evaluate(ctx, one)
        e1.record()
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
    res = {"params": pname, "special_primes": len(p.special), "keyswitch_digits": ks_shape(p.L, len(p.special))[0],
           "inferences_per_s": round(B * steps / elapsed, 2), "ms_per_step": round(elapsed / steps * 1e3, 3),
           "latency_p50_ms": round(float(np.percentile(lat, 50)), 3),
           "keyswitch_us_per_job": whole and whole["us_per_job"],
           "keyswitch_us_per_job_by_kernel": whole and whole["us_per_job_by_kernel"],
           "keyswitch_valu_frac": whole and whole["valu_frac"],
           "inner_kernel_valu_frac": inner_frac and round(inner_frac, 4),
           "inner_kernel_ops_per_job": ks_inner_ops(p.N, p.L, len(p.special)), "decrypted": B}
    del reqs, keys, plan, ctx
    torch.cuda.empty_cache()
    return res


def _plain_logits_mod_t(img, w, t):
    """The network on plaintext integers, reduced mod t after every layer:
    5x5 stride-2 convolution over the image zero-padded to 29x29, square,
    dense 845 -> 100, square, dense 100 -> 10."""
    import numpy as np
    pad = np.zeros((29, 29), dtype=np.int64)
    pad[:28, :28] = img
    win = np.lib.stride_tricks.sliding_window_view(pad, (5, 5))[::2, ::2]      # [13][13][5][5]
    conv = np.einsum("yxij,mij->myx", win, w.conv_w.astype(np.int64)) + w.conv_b.astype(np.int64)[:, None, None]
    a1 = (conv % t) ** 2 % t
    h = (w.w1.astype(np.int64) @ a1.reshape(845) + w.b1.astype(np.int64)) % t
    return (w.w2.astype(np.int64) @ (h * h % t) + w.b2.astype(np.int64)) % t


def cpu_baseline(p, w, recipe):
    """The oracle on the host cores: one full MNIST-shaped inference on
    ciphertexts with the schedule of the timed plan's recipe ("full" or
    "shared"; keys and encrypted inputs prepared outside the timing)."""
    from oracle import bfv
    from oracle import network as nw
    from paper_1812_10659_amd import workloads as wl
    octx = bfv.Context(p)
    sched = nw.mnist_schedule(w, recipe=recipe)
    keys = bfv.keygen(octx, wl.key_seed(1), nw.galois_elements(sched))
    img = wl.mnist_image(index=0)
    ins = nw.mnist_inputs(img)
    cts = [bfv.encrypt(octx, keys, bfv.encode(octx, nw.dense_slots(m, p.N, p.t)), 1, i) for i, m in enumerate(ins)]
    t0 = time.perf_counter()
    nw.run_ciphertexts(octx, keys, sched, cts)
    dt = time.perf_counter() - t0
    return {"value": round(1.0 / dt, 5), "unit": "inferences/s", "cores": bfv.max_threads(), "kind": "oracle",
            "sample": f"1 full inference, the timed plan's schedule ({sched.count('rotate')} rotations, "
                      f"{sched.count('square')} squares), {dt:.1f} s",
            "cpu": _cpu_model(), "batched_primitives_per_op": oracle_batch_ops()}


def cpu_baseline_full(workloads=("cfg0", "cfg1", "cfg3d", "cfg3s"), threads=("all", "1")):
    """The oracle on whole workloads, on all host threads and on one: the
    dense-64 query at N=4096, the MNIST-shaped network (the timed plan's
    shared-reduction schedule), and the transfer head at N=16384 in both
    recipes (dense row major, 4 queries per message, 3407 rotations; stacked
    row major, one query, 911 rotations).  Per workload and thread count:
    key generation, encryption of the inputs, the evaluation, decryption and
    decoding, each timed; the decrypted results are checked against the plain
    network.  Progress goes to stderr as the evaluation proceeds."""
    import numpy as np

    from oracle import bfv
    from oracle import network as nw
    from paper_1812_10659_amd import workloads as wl
    x64, W64 = wl.dense64_inputs()
    mw, img = wl.mnist_weights(), wl.mnist_image(index=0)
    hw, hf = wl.head_weights(), wl.head_features(4)
    cases = [
        ("cfg0", "cfg0 dense-64 query, N=4096, L=3", "n4096_3q", nw.dense64_schedule(W64), nw.dense64_inputs(x64, 4096),
         list(nw._mod(nw.dense64_plain(x64, W64), wl.PARAMS["n4096_3q"].t)), 1),
        ("cfg1", "cfg1 MNIST-shaped, N=16384, L=7 (shared reduction, 58 rotations)", "mnist_n16384",
         nw.mnist_schedule(mw, recipe="shared"), nw.mnist_inputs(img),
         list(nw._mod(nw.mnist_plain(img, mw), wl.PARAMS["mnist_n16384"].t)), 1),
        ("cfg3d", "cfg3 transfer head, N=16384, L=6, dense row major (4 queries per message)", "head_n16384",
         nw.head_schedule(hw), nw.head_inputs(hf),
         list(nw._mod(np.concatenate([nw.head_plain(hf[q], hw) for q in range(4)]), wl.PARAMS["head_n16384"].t)), 4),
        ("cfg3s", "cfg3 transfer head, N=16384, L=6, stacked row major (1 query per message)", "head_n16384",
         nw.head_stacked_schedule(hw), nw.head_stacked_inputs(hf[:1]),
         list(nw._mod(nw.head_plain(hf[0], hw), wl.PARAMS["head_n16384"].t)), 1),
    ]
    all_threads = bfv.max_threads()
    out = {"cpu": _cpu_model(), "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
           "kind": "oracle", "runs": []}
    for th in [all_threads if x == "all" else int(x) for x in threads]:
        bfv.set_threads(th)
        for key, name, pname, sched, ins, expected, queries in cases:
            if key not in workloads:
                continue
            p = wl.PARAMS[pname]
            octx = bfv.Context(p)
            t0 = time.perf_counter()
            keys = bfv.keygen(octx, 77, nw.galois_elements(sched))
            t1 = time.perf_counter()
            cts = [bfv.encrypt(octx, keys, bfv.encode(octx, nw.dense_slots(m, p.N, p.t)), 5, i)
                   for i, m in enumerate(ins)]
            t2 = time.perf_counter()

            def progress(done, total, name=name, th=th):
                print(f"[cpu-baseline] {name}, {th} threads: {done}/{total} ops", file=sys.stderr, flush=True)
            outs, _ = nw.run_ciphertexts(octx, keys, sched, cts, progress=progress)
            t3 = time.perf_counter()
            slots = [bfv.decode(octx, bfv.decrypt(octx, keys, o)) for o in outs]
            t4 = time.perf_counter()
            # the labelled result slots hold the network's outputs (compared as
            # a multiset: the labels order them per schedule)
            got = sorted(int(o_slots[s]) for o_slots, where in zip(slots, sched.out_slots) for s in where)
            ok = got == sorted(int(v) for v in expected)
            run = {"workload": name, "threads": th, "rotations": sched.count("rotate"),
                   "squares": sched.count("square"), "mul_plain": sched.count("mul_plain"), "queries": queries,
                   "keygen_s": round(t1 - t0, 3), "encrypt_s": round(t2 - t1, 3), "evaluate_s": round(t3 - t2, 3),
                   "decrypt_s": round(t4 - t3, 3), "inferences_per_s": round(queries / (t3 - t2), 5),
                   "client_inclusive_inferences_per_s": round(queries / (t4 - t1), 5), "decrypts_to_network": ok}
            print(f"[cpu-baseline] {json.dumps(run)}", file=sys.stderr, flush=True)
            out["runs"].append(run)
    bfv.set_threads(all_threads)
    return out


def oracle_batch_ops():
    """The oracle's per-operation times at the batched-primitive shape
    (N=16384, L=8), on all host threads and on one, and the batch's time
    extrapolated from them (512 mul_plain, 256 mul + relin and the batch's
    uneven rotation chains; not measured as a whole)."""
    import numpy as np

    from oracle import bfv
    from paper_1812_10659_amd import workloads as wl
    p = wl.PARAMS["batch_n16384_k2"]
    octx = bfv.Context(p)
    keys = bfv.keygen(octx, wl.key_seed(2), [bfv.galois_element(p.N, 1)])
    rs = wl.rng(wl.workload_seed(2), 21)
    m1, m2 = (rs.integers(0, p.t, p.N).astype(np.uint64) for _ in range(2))
    c1, c2 = bfv.encrypt(octx, keys, m1, 1, 1), bfv.encrypt(octx, keys, m2, 1, 2)
    all_threads = bfv.max_threads()

    def timed(f, *a):
        t0 = time.perf_counter()
        r = f(*a)
        return time.perf_counter() - t0, r

    per = {}
    for th in sorted({all_threads, 1}, reverse=True):
        bfv.set_threads(th)
        t_mp, _ = timed(bfv.mul_plain, octx, c1, m2)
        t_mul, c3 = timed(bfv.mul, octx, c1, c2)
        t_rl, _ = timed(bfv.relin, octx, c3, keys.rlk)
        t_rot, _ = timed(bfv.rotate, octx, c1, 1, keys)
        per[f"threads_{th}"] = {"mul_plain_s": round(t_mp, 4), "mul_s": round(t_mul, 4), "relin_s": round(t_rl, 4),
                                "rotate_s": round(t_rot, 4)}
    bfv.set_threads(all_threads)
    a = per[f"threads_{all_threads}"]
    rot = int(wl.batch_rotation_counts(512).sum())
    est = 512 * a["mul_plain_s"] + 256 * (a["mul_s"] + a["relin_s"]) + rot * a["rotate_s"]
    return {"config": "N=16384, L=8 (the batched-primitive shape)", **per,
            "extrapolated_batch_s": round(est, 1),
            "extrapolated_note": f"512 mul_plain + 256 (mul + relin) + {rot} rotations at the all-thread per-op "
                                 f"times; extrapolated, not measured"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
