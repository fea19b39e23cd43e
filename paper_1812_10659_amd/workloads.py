"""Parameter sets and seeded synthetic inputs.

This module is the only thing the GPU library's callers and the CPU oracle
share.  It holds numbers and random-number recipes, none of the scheme's
arithmetic: prime lists are plain constants, and every generator only draws
seeded numpy values of the shapes the paper's workloads have.

Prime choice: the ciphertext primes are the largest primes below 2^30 that are
congruent to 1 modulo 2N (so a negacyclic NTT of length N exists, the same
condition the paper states for slot batching mod p in Sec. 3.1).  The plaintext
modulus t is a prime congruent to 1 modulo 2N, so that R_t splits into N slots.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List

import numpy as np

# Largest primes q < 2^30 with q = 1 (mod 2N), in decreasing order.
PRIMES_4096 = [1073692673, 1073668097, 1073651713, 1073643521, 1073569793,
               1073479681, 1073430529, 1073299457]
PRIMES_16384 = [1073643521, 1073479681, 1073184769, 1073053697, 1072857089,
                1072496641, 1071513601, 1071415297, 1071087617, 1070727169,
                1070432257, 1069219841, 1068564481, 1068466177]

# Classical 128-bit security caps on log2(Q*P) for a ternary secret, per ring
# degree (the homomorphic-encryption security standard's table).
SECURITY_CAP_LOG2 = {1024: 27, 2048: 54, 4096: 109, 8192: 218, 16384: 438, 32768: 881}


@dataclasses.dataclass(frozen=True)
class ParamSet:
    name: str
    N: int
    t: int
    q: tuple          # ciphertext (data) primes q_0..q_{L-1}
    P: int            # special prime used by key switching
    insecure_ok: bool = False   # toy sets for tests only
    P2: int = 0       # second special prime: key-switching digits of two primes

    @property
    def L(self) -> int:
        return len(self.q)

    @property
    def special(self) -> tuple:
        return (self.P, self.P2) if self.P2 else (self.P,)


PARAMS: Dict[str, ParamSet] = {
    # N=4096, t=65537 with two 30-bit primes (q ~ 2^60) as first specified.
    # The oracle's noise check shows the square activation does not fit in it.
    "n4096_2q": ParamSet("n4096_2q", 4096, 65537, tuple(PRIMES_4096[:2]), PRIMES_4096[2]),
    # N=4096 working set: three 30-bit primes and a 19-bit special prime,
    # log2(QP) = 108.7 <= 109.
    "n4096_3q": ParamSet("n4096_3q", 4096, 65537, tuple(PRIMES_4096[:3]), 417793),
    # MNIST-shaped network, N=16384, t ~ 2^20.13, seven data primes.
    "mnist_n16384": ParamSet("mnist_n16384", 16384, 1146881, tuple(PRIMES_16384[:7]), PRIMES_16384[7]),
    # The same ciphertext primes with key-switching digits of two primes and
    # two special primes: 4 digits instead of 7, log2(QP) = 270 <= 438.
    "mnist_n16384_k2": ParamSet("mnist_n16384_k2", 16384, 1146881, tuple(PRIMES_16384[:7]), PRIMES_16384[7],
                                P2=PRIMES_16384[8]),
    # Batched primitive microbenchmark: eight data primes.
    "batch_n16384": ParamSet("batch_n16384", 16384, 1146881, tuple(PRIMES_16384[:8]), PRIMES_16384[8]),
    "batch_n16384_k2": ParamSet("batch_n16384_k2", 16384, 1146881, tuple(PRIMES_16384[:8]), PRIMES_16384[8],
                                P2=PRIMES_16384[9]),
    # LoLa-Dense input path: the mask products at the input cost noise that
    # seven data primes do not leave room for; eight primes, log2(QP) = 270.
    "mnist_dense_n16384": ParamSet("mnist_dense_n16384", 16384, 1146881, tuple(PRIMES_16384[:8]), PRIMES_16384[8]),
    # CIFAR-shaped network: the same noise demand (seven primes leave no
    # budget after the second convolution's one-hot products); eight primes.
    "cifar_n16384": ParamSet("cifar_n16384", 16384, 1146881, tuple(PRIMES_16384[:8]), PRIMES_16384[8]),
    # A convolution front end followed by a longer dense chain (three squares
    # after the convolution's, each row-major layer's products on top): ten
    # data primes, log2(QP) = 330 <= 438.
    "chain_n16384": ParamSet("chain_n16384", 16384, 1146881, tuple(PRIMES_16384[:10]), PRIMES_16384[10]),
    # The LoLa-Dense and CIFAR-shaped sets with key-switching digits of two
    # primes and two special primes (log2(QP) = 300 <= 438).
    "mnist_dense_n16384_k2": ParamSet("mnist_dense_n16384_k2", 16384, 1146881, tuple(PRIMES_16384[:8]),
                                      PRIMES_16384[8], P2=PRIMES_16384[9]),
    "cifar_n16384_k2": ParamSet("cifar_n16384_k2", 16384, 1146881, tuple(PRIMES_16384[:8]), PRIMES_16384[8],
                                P2=PRIMES_16384[9]),
    # Transfer-learning head: six data primes.
    "head_n16384": ParamSet("head_n16384", 16384, 1146881, tuple(PRIMES_16384[:6]), PRIMES_16384[6]),
    "head_n16384_k2": ParamSet("head_n16384_k2", 16384, 1146881, tuple(PRIMES_16384[:6]), PRIMES_16384[6],
                               P2=PRIMES_16384[7]),
    # The largest ciphertext-prime count the library accepts: twelve data
    # primes (log2(QP) = 390 <= 438), for tests at that limit.
    "l12_n16384": ParamSet("l12_n16384", 16384, 1146881, tuple(PRIMES_16384[:12]), PRIMES_16384[12]),
    # The same with two special primes: six digits of two primes, fourteen
    # key-switching moduli (log2(QP) = 420 <= 438), the largest shape the
    # library accepts with digits of two primes.
    "l12_n16384_k2": ParamSet("l12_n16384_k2", 16384, 1146881, tuple(PRIMES_16384[:12]), PRIMES_16384[12],
                              P2=PRIMES_16384[13]),
    # N=8192 for tests of that ring size: five data primes, log2(QP) = 180 <= 218.
    "n8192": ParamSet("n8192", 8192, 65537, tuple(PRIMES_16384[:5]), PRIMES_16384[5]),
    # Small sets for tests (not secure; flagged).
    # (primes = 1 mod 2^15 are also = 1 mod 2N for these smaller N)
    "toy1024": ParamSet("toy1024", 1024, 12289, tuple(PRIMES_16384[:3]), PRIMES_16384[3],
                        insecure_ok=True),
    "toy2048": ParamSet("toy2048", 2048, 40961, tuple(PRIMES_16384[:4]), PRIMES_16384[4],
                        insecure_ok=True),
    "toy1024_k2": ParamSet("toy1024_k2", 1024, 12289, tuple(PRIMES_16384[:3]), PRIMES_16384[3],
                           insecure_ok=True, P2=PRIMES_16384[4]),
    # one ciphertext prime with two special primes: a single digit holding
    # fewer primes than the special primes (words only; the noise of a product
    # exceeds this Delta, so the network checks do not use it)
    "toy1024_l1_k2": ParamSet("toy1024_l1_k2", 1024, 12289, tuple(PRIMES_16384[:1]), PRIMES_16384[1],
                              insecure_ok=True, P2=PRIMES_16384[2]),
}

# Plaintext moduli for exact integer outputs of the MNIST-shaped network by
# CRT: primes t = 1 mod 2N (N = 16384), product 2^132.7 above twice the
# network's worst-case |logit| (2^119.6 for the seeded weights), each leaving
# a positive noise budget after the whole network at seven data primes
# (t = 1769473, 2424833 and larger were measured to exhaust it).
MNIST_CRT_T = (65537, 163841, 557057, 786433, 1146881, 1179649, 1376257)


def crt_params(base: str = "mnist_n16384", moduli=MNIST_CRT_T) -> List[ParamSet]:
    """One parameter set per plaintext modulus, ciphertext primes of `base`."""
    b = PARAMS[base]
    return [dataclasses.replace(b, name=f"{base}_t{t}", t=int(t)) for t in moduli]


MASTER_SEED = 1812106590


# Workload ids: 0 dense-64 query (N=4096), 1 MNIST-shaped network (N=16384),
# 2 batched primitives (N=16384, eight primes), 3 transfer-learning head
# (N=16384), 4 mixed serving stream.
DENSE64, MNIST, BATCH, HEAD, SERVE = 0, 1, 2, 3, 4


def workload_seed(k: int) -> int:
    """Master seed of workload k."""
    return MASTER_SEED + k


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """A numpy generator for (seed, stream): streams separate keys, data, weights."""
    return np.random.Generator(np.random.PCG64([seed, stream]))


# Stream ids inside a workload's seed.
STREAM_KEYS, STREAM_ENC, STREAM_DATA, STREAM_WEIGHTS, STREAM_ARRIVALS = 1, 2, 3, 4, 5


def key_seed(k: int) -> int:
    return int(rng(workload_seed(k), STREAM_KEYS).integers(0, 2**63))


def enc_seed(k: int) -> int:
    return int(rng(workload_seed(k), STREAM_ENC).integers(0, 2**63))


# -------------------------------------------------------------- dense-64 query, N=4096
def dense64_inputs(seed: int | None = None):
    """64-vector x and 64x64 matrix W, both uniform int8."""
    s = workload_seed(0) if seed is None else seed
    x = rng(s, STREAM_DATA).integers(-128, 128, size=64).astype(np.int64)
    W = rng(s, STREAM_WEIGHTS).integers(-128, 128, size=(64, 64)).astype(np.int64)
    return x, W


# -------------------------------------------------------------- MNIST-shaped network, N=16384
@dataclasses.dataclass
class MnistWeights:
    conv_w: np.ndarray   # [5 maps][5][5] int8 values
    conv_b: np.ndarray   # [5] int32 values
    w1: np.ndarray       # [100][845] int8, input index 169*map + 13*y + x
    b1: np.ndarray       # [100]
    w2: np.ndarray       # [10][100]
    b2: np.ndarray       # [10]


def mnist_image(seed: int | None = None, index: int = 0) -> np.ndarray:
    """A 28x28 image with uniform values 0..255."""
    s = workload_seed(1) if seed is None else seed
    return rng(s, STREAM_DATA * 1000 + index).integers(0, 256, size=(28, 28)).astype(np.int64)


def mnist_weights(seed: int | None = None) -> MnistWeights:
    s = workload_seed(1) if seed is None else seed
    g = rng(s, STREAM_WEIGHTS)
    conv_w = g.integers(-128, 128, size=(5, 5, 5)).astype(np.int64)
    conv_b = g.integers(-2**15, 2**15, size=5).astype(np.int64)
    w1 = g.integers(-128, 128, size=(100, 845)).astype(np.int64)
    b1 = g.integers(-2**15, 2**15, size=100).astype(np.int64)
    w2 = g.integers(-128, 128, size=(10, 100)).astype(np.int64)
    b2 = g.integers(-2**15, 2**15, size=10).astype(np.int64)
    return MnistWeights(conv_w, conv_b, w1, b1, w2, b2)


@dataclasses.dataclass
class MnistSmallWeights:
    conv_w: np.ndarray   # [5 maps][5][5] int8 values (those of the MNIST-shaped network)
    conv_b: np.ndarray   # [5]
    w: np.ndarray        # [10][845] int8, input index 169*map + 13*y + x
    b: np.ndarray        # [10]


def mnist_small_weights(seed: int | None = None) -> MnistSmallWeights:
    """The small variant: the MNIST-shaped network's convolution, then one
    dense layer 845 -> 10 with its own seeded weights."""
    s = workload_seed(1) if seed is None else seed
    big = mnist_weights(s)
    g = rng(s, STREAM_WEIGHTS * 10 + 1)
    w = g.integers(-128, 128, size=(10, 845)).astype(np.int64)
    b = g.integers(-2**15, 2**15, size=10).astype(np.int64)
    return MnistSmallWeights(big.conv_w, big.conv_b, w, b)


# ----------------------------------------------- CIFAR-shaped network, N=16384
@dataclasses.dataclass
class CifarWeights:
    conv1_w: np.ndarray   # [m1][3][8][8] int8 values
    conv1_b: np.ndarray   # [m1]
    conv2_w: np.ndarray   # [m2][m1][6][6] int8 values
    conv2_b: np.ndarray   # [m2]
    w3: np.ndarray        # [10][m2*v2] int8, input index v2*map + n2*y + x (v2 = n2^2 = 25)
    b3: np.ndarray        # [10]


def cifar_image(seed: int | None = None, index: int = 0) -> np.ndarray:
    """A 3x32x32 image with uniform values 0..255."""
    s = workload_seed(5) if seed is None else seed
    return rng(s, STREAM_DATA * 1000 + index).integers(0, 256, size=(3, 32, 32)).astype(np.int64)


def cifar_weights(seed: int | None = None, m1: int = 83, m2: int = 163, v2: int = 25) -> CifarWeights:
    """The collapsed CIFAR network's shapes (8x8x3 convolution, 83 maps;
    6x6x83 convolution, 163 maps; dense 4075 -> 10) with seeded int8
    weights; m1 and m2 shrink the map counts and v2 (outputs per map of the
    second convolution) the dense layer for small test cases."""
    s = workload_seed(5) if seed is None else seed
    g = rng(s, STREAM_WEIGHTS)
    c1w = g.integers(-128, 128, size=(83, 3, 8, 8)).astype(np.int64)[:m1]
    c1b = g.integers(-2**15, 2**15, size=83).astype(np.int64)[:m1]
    c2w = g.integers(-128, 128, size=(163, 83, 6, 6)).astype(np.int64)[:m2, :m1]
    c2b = g.integers(-2**15, 2**15, size=163).astype(np.int64)[:m2]
    w3 = g.integers(-128, 128, size=(10, 163 * 25)).astype(np.int64)[:, :m2 * v2]
    b3 = g.integers(-2**15, 2**15, size=10).astype(np.int64)
    return CifarWeights(c1w, c1b, c2w, c2b, w3, b3)


# -------------------------------------------------------------- batched primitives, N=16384
def batch_rotation_counts(n_ct: int = 512, seed: int | None = None) -> np.ndarray:
    """Per-ciphertext rotation counts, uniform in 1..64 (uneven on purpose)."""
    s = workload_seed(2) if seed is None else seed
    return rng(s, STREAM_DATA * 10 + 1).integers(1, 65, size=n_ct).astype(np.int64)


def batch_rotation_steps(counts: np.ndarray, N: int = 16384, seed: int | None = None) -> List[np.ndarray]:
    """Rotation steps per ciphertext, uniform over {+2^j : 2^j < N/2} plus the
    row swap (encoded as 0)."""
    s = workload_seed(2) if seed is None else seed
    g = rng(s, STREAM_DATA * 10 + 2)
    choices = [1 << j for j in range(int(np.log2(N // 2)))] + [0]
    return [np.array([choices[i] for i in g.integers(0, len(choices), size=int(c))], dtype=np.int64)
            for c in counts]


def uniform_residues(n_polys: int, moduli, N: int, seed: int, stream: int) -> np.ndarray:
    """Uniform residues, shape [n_polys][len(moduli)][N], each limb mod its prime."""
    g = rng(seed, stream)
    out = np.empty((n_polys, len(moduli), N), dtype=np.uint32)
    for j, m in enumerate(moduli):
        out[:, j, :] = g.integers(0, m, size=(n_polys, N), dtype=np.uint64).astype(np.uint32)
    return out


# -------------------------------------------------------------- transfer-learning head, N=16384
@dataclasses.dataclass
class HeadWeights:
    w1: np.ndarray   # [256][4096] int8
    b1: np.ndarray   # [256]
    w2: np.ndarray   # [10][256] int8
    b2: np.ndarray   # [10]


def head_features(n_queries: int = 16, seed: int | None = None) -> np.ndarray:
    """Feature vectors: clip(round(N(0, 20^2)), -128, 127), dimension 4096."""
    s = workload_seed(3) if seed is None else seed
    f = rng(s, STREAM_DATA).normal(0.0, 20.0, size=(n_queries, 4096))
    return np.clip(np.rint(f), -128, 127).astype(np.int64)


def head_weights(seed: int | None = None) -> HeadWeights:
    s = workload_seed(3) if seed is None else seed
    g = rng(s, STREAM_WEIGHTS)
    w1 = g.integers(-128, 128, size=(256, 4096)).astype(np.int64)
    b1 = g.integers(-2**15, 2**15, size=256).astype(np.int64)
    w2 = g.integers(-128, 128, size=(10, 256)).astype(np.int64)
    b2 = g.integers(-2**15, 2**15, size=10).astype(np.int64)
    return HeadWeights(w1, b1, w2, b2)


# -------------------------------------------------------------- serving mix
def serving_arrivals(n_req: int = 2000, rate: float = 200.0, p_large: float = 0.7,
                  seed: int | None = None):
    """Poisson arrival times (s) and request kinds (1 = N=16384 MNIST-shaped,
    0 = N=4096 dense-64 query)."""
    s = workload_seed(4) if seed is None else seed
    g = rng(s, STREAM_ARRIVALS)
    gaps = g.exponential(1.0 / rate, size=n_req)
    kinds = (g.random(n_req) < p_large).astype(np.int64)
    return np.cumsum(gaps), kinds
