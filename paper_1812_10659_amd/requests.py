"""Client-side set-up of request batches: key sets and encrypted inputs made
through the library, packed with a plan's input map.  Marshalling only: every
key, encryption and evaluation runs in the library's kernels."""
from __future__ import annotations

import numpy as np

from . import networks
from . import workloads as wl


def client_keys(ctx, plan, n_clients: int, base_seed: int, stride: int = 7919):
    """n_clients key sets (secret, public, relinearisation and the plan's
    Galois keys); client c's seed is base_seed + stride * c."""
    keys = []
    gal = plan.galois()
    for c in range(n_clients):
        ks = base_seed + stride * c
        sk = ctx.keygen_secret(ks)
        keys.append(dict(seed=ks, sk=sk, pk=ctx.keygen_public(ks, sk), rlk=ctx.keygen_switch(ks, sk, 0),
                         gks=[ctx.keygen_switch(ks, sk, g) for g in gal]))
    return keys


def encrypted_request(ctx, plan, key, values, enc_seed: int):
    """One request: the values packed into the plan's input messages,
    encrypted under the key set with encryption seed enc_seed (message i takes
    object id i), and empty output ciphertexts."""
    msgs = networks.pack_inputs(plan.input_map(), values)
    ins = [ctx.encrypt(key["pk"], ctx.encode(m), enc_seed, i) for i, m in enumerate(msgs)]
    return dict(rlk=key["rlk"], gks=key["gks"], inputs=ins,
                outputs=[ctx.empty_ct() for _ in range(plan.info["n_outputs"])])


def mnist_batch(ctx, plan, n_requests: int, n_clients: int):
    """The MNIST-shaped batch the benchmark times: request r is seeded image r,
    under key set r mod n_clients (key seeds key_seed(1) + 7919 c), encrypted
    with seed enc_seed(1) + r.  Returns (requests, keys, images)."""
    C = max(1, min(n_clients, n_requests))
    keys = client_keys(ctx, plan, C, wl.key_seed(1))
    reqs, images = [], []
    for r in range(n_requests):
        img = wl.mnist_image(index=r)
        images.append(img)
        reqs.append(encrypted_request(ctx, plan, keys[r % C], networks.mnist_input_values(img), wl.enc_seed(1) + r))
    return reqs, keys, images


def decrypted_outputs(ctx, plan, sk, request) -> np.ndarray:
    """The request's result values: its output messages decrypted, decoded
    and read with the plan's output map."""
    slots = np.stack([ctx.decode(ctx.decrypt(sk, o)) for o in request["outputs"]])
    return networks.unpack_outputs(plan.output_map(), slots)
