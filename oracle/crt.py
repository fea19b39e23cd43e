"""Exact integers from residues modulo several plaintext moduli (oracle side).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A network whose outputs exceed one plaintext modulus t is run once per
modulus t_i of a pairwise coprime set, and the outputs mod t_i are combined by
the Chinese remainder theorem (Sec. 4.4 runs its CIFAR network under three
plaintext moduli).  The combination is exact when M = prod t_i exceeds twice
the largest magnitude the outputs can take, which `mnist_logit_bound` gives
for the MNIST-shaped network from its actual weights.

Written as the textbook reconstruction X = sum_i r_i M_i (M_i^-1 mod t_i) mod M
(M_i = M / t_i) on Python integers, centred into [-M/2, M/2).
"""
from __future__ import annotations

from math import gcd, prod
from typing import Sequence


def crt_combine(residues: Sequence[int], moduli: Sequence[int]) -> int:
    """The integer X in [-M/2, M/2) with X = residues[i] mod moduli[i]."""
    if len(residues) != len(moduli) or not moduli:
        raise ValueError("one residue per modulus")
    for i, a in enumerate(moduli):
        for b in moduli[:i]:
            if gcd(a, b) != 1:
                raise ValueError("moduli must be pairwise coprime")
    M = prod(moduli)
    x = 0
    for r, t in zip(residues, moduli):
        Mi = M // t
        x += int(r) * Mi * pow(Mi, -1, t)
    x %= M
    return x - M if x >= (M + 1) // 2 else x


def mnist_logit_bound(wts, pixel_max: int = 255) -> int:
    """An upper bound on |logit| of the MNIST-shaped network (5x5 convolution
    over pixels in [0, pixel_max] -> square -> dense -> square -> dense), from
    the magnitudes of its weights and biases."""
    conv = max(pixel_max * sum(abs(int(v)) for v in wts.conv_w[m].reshape(-1)) + abs(int(wts.conv_b[m]))
               for m in range(wts.conv_w.shape[0]))
    a1 = conv * conv
    h = max(sum(abs(int(v)) for v in row) * a1 + abs(int(b)) for row, b in zip(wts.w1, wts.b1))
    a2 = h * h
    return max(sum(abs(int(v)) for v in row) * a2 + abs(int(b)) for row, b in zip(wts.w2, wts.b2))
