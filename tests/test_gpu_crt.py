"""GPU parity of exact integer outputs by CRT over several plaintext moduli:
the device combination against the oracle's reconstruction, and the
MNIST-shaped network's integer logits against the exact integer network."""
import math
import random

import numpy as np
import pytest

from oracle import crt as ocrt
from oracle import network as nw
from paper_1812_10659_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mods,words", [((65537,), 1), ((3, 5, 7), 1), ((557057, 786433, 1146881), 2),
                                        (wl.MNIST_CRT_T, 3), (wl.MNIST_CRT_T, 4)])
def test_crt_combine_matches_oracle(mods, words):
    import torch
    from paper_1812_10659_amd import crt
    print(f"[gpu-crt] combine k={len(mods)} words={words}", flush=True)
    M = math.prod(mods)
    rng = random.Random(len(mods) * 10 + words)
    xs = [rng.randrange(-(M // 2), (M + 1) // 2) for _ in range(997)]
    xs += [-(M // 2), (M - 1) // 2, 0, 1, -1, M // 3, -(M // 3)]
    # residues as the decoder gives them ([0, t)) and as arbitrary representatives
    res = [torch.tensor([x % t for x in xs], dtype=torch.int64, device="cuda") for t in mods]
    res[0] = res[0] - mods[0] * (torch.arange(len(xs), device="cuda") % 3)
    got = crt.words_to_ints(crt.crt_combine(res, mods, words).cpu().numpy())
    exp = [ocrt.crt_combine([x % t for t in mods], mods) for x in xs]
    assert exp == xs and got == exp


def test_crt_combine_rejects_bad_arguments():
    import torch
    from paper_1812_10659_amd import crt, lola
    r = [torch.zeros(4, dtype=torch.int64, device="cuda")] * 2
    with pytest.raises(lola.LolaError):
        crt.crt_combine(r, (6, 9), 1)                      # not coprime
    with pytest.raises(lola.LolaError):
        crt.crt_combine([r[0]] * 7, wl.MNIST_CRT_T, 2)     # 2^132.7 does not fit 128 bits
    with pytest.raises(lola.LolaError):
        crt.crt_combine(r, (65537, 1 << 27), 2)            # modulus out of range


def test_integer_logits_equal_the_network():
    """Seven plaintext moduli, each a full encrypted evaluation; the combined
    logits equal the exact integer network (no reduction mod t)."""
    import torch
    from paper_1812_10659_amd import crt, networks
    print("[gpu-crt] MNIST-shaped network under 7 plaintext moduli", flush=True)
    w = wl.mnist_weights()
    net = crt.CrtNetwork(wl.crt_params(), networks.mnist_layers(w))
    keys = net.keygen(wl.key_seed(1) + 17)
    imgs = [wl.mnist_image(index=i) for i in (0, 5)]
    reqs = [net.request(keys, networks.mnist_input_values(img), 40 + k) for k, img in enumerate(imgs)]
    net.evaluate(reqs)
    torch.cuda.synchronize()
    for img, req in zip(imgs, reqs):
        got = net.integers(keys, req)
        exp = [int(v) for v in nw.mnist_plain(img, w)]
        assert got == exp
        assert max(abs(v) for v in exp) > max(wl.MNIST_CRT_T) ** 3   # far beyond one modulus
