"""BFV reference scheme (the oracle).

TEST INFRASTRUCTURE ONLY: the slow, plainly written CPU reference that the GPU
library is checked against.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU library; the
polynomial arithmetic comes from oracle/bfv_ref.c and every multi-precision
step (CRT lifts, exact rounding) uses Python integers.

What is computed (the paper fixes the scheme's interface in Sec. 3.1: E, D,
the homomorphic + and x, message-times-scalar products from Sec. 4.2.2, and
the row-swap / column-rotation operations on the 2 x N/2 slot matrix):

  ring      R_m = Z_m[X]/(X^N+1); polynomials are numpy uint64 arrays of
            residues, shape [L][N] (one row per prime), coefficient form.
  Q         q_0 * ... * q_{L-1};  Delta = floor(Q / t).
  slots     slot (r, i), r in {0,1}, i < N/2, of m in R_t is m(zeta^e(r,i)) with
            e(r,i) = (2N-1)^r * 3^i mod 2N and zeta the smallest g with
            g^N = -1 (mod t)  (Sec. 3.1: a 2N-th root of unity mod p makes R_p
            a vector of N slots).
  rotate    rotate(+k) = automorphism X -> X^(3^k mod 2N): output slot (r,i)
            takes input slot (r, i+k mod N/2) (a left rotation of each row);
            the row swap uses X -> X^(2N-1).  The paper's rotation "by k to the
            right" is rotate(-k).
  keys      s ternary; pk = (-(a s + e), a) mod Q; a key-switching key for a
            target s' is, for each digit d and each modulus m in
            {q_0..q_{L-1}, p_0..p_{K-1}}:
            b_d = -a_d s + e_d + [m is a prime of digit d] (P mod m) s',
            a_d uniform, P = p_0 ... p_{K-1}.
  encrypt   c = (pk0 u + e1 + Delta m, pk1 u + e2) mod Q.
  decrypt   x = c0 + c1 s (+ c2 s^2) mod Q lifted to [0,Q); m_k = round(t x_k/Q) mod t.
  mul       exact: lift the four inputs to centred integers, take the three
            negacyclic tensor products over Z, then round(t d_j / Q) mod Q.
  keyswitch hybrid key switching with K special primes and digits of K
            consecutive ciphertext primes (the last may hold fewer): digit d
            of modulus Q_d (the product of its primes) is D_d = x mod Q_d in
            [0, Q_d); u = sum_d D_d * ksk_d modulo every q_j and p_k; result
            (u - [u mod P]_P) / P mod q_j with [.]_P centred.  K = 1 gives
            one digit per prime.  The gadget P (Q/Q_d) ((Q/Q_d)^-1 mod Q_d)
            that digit d's key carries is P mod q_j at its own primes and 0
            at every other modulus, so sum_d D_d gadget_d = P x mod QP.

Every random value is drawn from ChaCha20 (RFC 8439) with
key = the 256-bit seed's eight words (least significant first), nonce =
(domain, object, limb), one 64-bit word per coefficient.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# ChaCha20 stream domains.
DOM_SK, DOM_PK_A, DOM_PK_E, DOM_KSK_A, DOM_KSK_E, DOM_ENC_U, DOM_ENC_E1, DOM_ENC_E2 = range(1, 9)

ROW_SWAP = "row_swap"

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build_oracle  # noqa: WPS433 (test infrastructure)
            build_oracle.build()
        L = ctypes.CDLL(_LIB_PATH)
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        c_u32, c_u64 = ctypes.c_uint32, ctypes.c_uint64
        L.or_min_root_2n.argtypes = [c_u64, c_u32]
        L.or_min_root_2n.restype = c_u64
        L.or_eval_odd.argtypes = [u64p, u64p, c_u32, c_u64, c_u64]
        L.or_interp_odd.argtypes = [u64p, u64p, c_u32, c_u64, c_u64]
        L.or_poly_mul_schoolbook.argtypes = [u64p, u64p, u64p, c_u32, c_u64]
        L.or_poly_mul.argtypes = [u64p, u64p, u64p, c_u32, c_u64]
        L.or_poly_mul_many.argtypes = [u64p, u64p, u64p, c_u32, u64p, c_u32]
        L.or_automorph.argtypes = [u64p, u64p, c_u32, c_u64, c_u64]
        L.or_chacha20_block.argtypes = [u32p, c_u32, u32p, u32p]
        L.or_stream_words.argtypes = [u32p, c_u32, c_u32, c_u32, c_u32, u64p]
        L.or_sample_uniform.argtypes = [u32p, c_u32, c_u32, c_u32, c_u32, c_u64, u64p]
        L.or_sample_ternary.argtypes = [u32p, c_u32, c_u32, c_u32, i64p]
        L.or_sample_cbd.argtypes = [u32p, c_u32, c_u32, c_u32, i64p]
        L.or_max_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)


# ------------------------------------------------------------ primitives --
def poly_mul(a, b, m: int) -> np.ndarray:
    """Negacyclic product mod m (transform-based)."""
    out = np.empty(len(a), np.uint64)
    lib().or_poly_mul(_u64(a), _u64(b), out, len(a), m)
    return out


def poly_mul_schoolbook(a, b, m: int) -> np.ndarray:
    """Negacyclic product mod m by its definition, O(N^2)."""
    out = np.empty(len(a), np.uint64)
    lib().or_poly_mul_schoolbook(_u64(a), _u64(b), out, len(a), m)
    return out


def poly_mul_many(pairs: Sequence) -> List[np.ndarray]:
    """[(a, b, m), ...] -> [a*b mod m, ...], independent products."""
    if not pairs:
        return []
    N = len(pairs[0][0])
    A = np.ascontiguousarray(np.stack([p[0] for p in pairs]).astype(np.uint64))
    B = np.ascontiguousarray(np.stack([p[1] for p in pairs]).astype(np.uint64))
    M = np.array([p[2] for p in pairs], dtype=np.uint64)
    out = np.empty_like(A)
    lib().or_poly_mul_many(A, B, out, N, M, len(pairs))
    return [out[i] for i in range(len(pairs))]


def automorph(a, m: int, g: int) -> np.ndarray:
    out = np.empty(len(a), np.uint64)
    lib().or_automorph(_u64(a), out, len(a), m, g)
    return out


def chacha20_block(key_words: Sequence[int], counter: int, nonce_words: Sequence[int]) -> np.ndarray:
    out = np.zeros(16, np.uint32)
    lib().or_chacha20_block(np.array(key_words, np.uint32), counter,
                            np.array(nonce_words, np.uint32), out)
    return out


def seed_key(seed: int) -> np.ndarray:
    """The ChaCha20 key of a seed: its eight 32-bit words, least significant
    first (seeds are integers in [0, 2^256); one below 2^64 leaves words 2..7
    zero)."""
    seed = int(seed)
    assert 0 <= seed < 1 << 256
    return np.array([(seed >> (32 * k)) & 0xFFFFFFFF for k in range(8)], np.uint32)


def stream_words(seed: int, domain: int, obj: int, limb: int, n: int) -> np.ndarray:
    out = np.empty(n, np.uint64)
    lib().or_stream_words(seed_key(seed), domain, obj, limb, n, out)
    return out


def sample_uniform(seed, domain, obj, limb, n, m) -> np.ndarray:
    out = np.empty(n, np.uint64)
    lib().or_sample_uniform(seed_key(seed), domain, obj, limb, n, m, out)
    return out


def sample_ternary(seed, domain, obj, n) -> np.ndarray:
    out = np.empty(n, np.int64)
    lib().or_sample_ternary(seed_key(seed), domain, obj, n, out)
    return out


def sample_cbd(seed, domain, obj, n) -> np.ndarray:
    out = np.empty(n, np.int64)
    lib().or_sample_cbd(seed_key(seed), domain, obj, n, out)
    return out


def min_root_2n(m: int, N: int) -> int:
    return int(lib().or_min_root_2n(m, N))


def set_threads(n: int) -> None:
    lib().or_set_threads(n)


def max_threads() -> int:
    return int(lib().or_max_threads())


# ------------------------------------------------------------ parameters --
class Context:
    """Derived constants of a parameter set (N, t, q_0..q_{L-1}, the special
    primes P and, when the set has one, P2)."""

    def __init__(self, params):
        self.params = params
        self.N = int(params.N)
        self.t = int(params.t)
        self.q = [int(x) for x in params.q]
        self.special = [int(params.P)] + ([int(params.P2)] if getattr(params, "P2", 0) else [])
        self.K = len(self.special)
        self.P = math.prod(self.special)
        self.L = len(self.q)
        self.Q = math.prod(self.q)
        self.delta = self.Q // self.t
        self.moduli = self.q + self.special
        # key-switching digits: K consecutive ciphertext primes each
        self.digits = [list(range(i, min(i + self.K, self.L))) for i in range(0, self.L, self.K)]
        self.zeta = min_root_2n(self.t, self.N)
        if self.zeta == 0:
            raise ValueError("t has no primitive 2N-th root")
        for m in self.moduli:
            if (m - 1) % (2 * self.N):
                raise ValueError(f"modulus {m} is not 1 mod 2N")
        # CRT reconstruction over Q: x = sum r_i * Qhat_i * (Qhat_i^-1 mod q_i) mod Q
        self._crt = [(self.Q // qi) * pow(self.Q // qi, -1, qi) for qi in self.q]
        # slot index -> evaluation index k, where the evaluation point is zeta^(2k+1)
        n2 = self.N // 2
        e = np.empty(self.N, dtype=np.int64)
        for r in range(2):
            base = (2 * self.N - 1) if r else 1
            for i in range(n2):
                e[r * n2 + i] = (base * pow(3, i, 2 * self.N)) % (2 * self.N)
        self.slot_exp = e
        self.slot_eval_index = (e - 1) // 2

    # --- integer views
    def crt_lift(self, limbs) -> np.ndarray:
        """[L][N] residues -> object array of integers in [0, Q)."""
        acc = np.zeros(self.N, dtype=object)
        for i, qi in enumerate(self.q):
            acc = acc + np.asarray(limbs[i], dtype=np.uint64).astype(object) * self._crt[i]
        return acc % self.Q

    def centred_lift(self, limbs) -> np.ndarray:
        x = self.crt_lift(limbs)
        half = self.Q // 2
        return np.where(x > half, x - self.Q, x)

    def reduce_int(self, x, moduli=None) -> np.ndarray:
        """Object (or int64) integer array -> [len(moduli)][N] residues."""
        moduli = self.q if moduli is None else moduli
        xo = np.asarray(x, dtype=object)
        return np.stack([np.array([int(v) % m for v in xo], dtype=np.uint64) for m in moduli])

    def small_to_limbs(self, v, moduli=None) -> np.ndarray:
        """Small signed int64 polynomial -> residues mod each modulus."""
        moduli = self.q if moduli is None else moduli
        v = np.asarray(v, dtype=np.int64)
        return np.stack([np.mod(v, m).astype(np.uint64) for m in moduli])


def galois_element(N: int, step) -> int:
    """Automorphism exponent g for rotate(step) (left by step within each row)
    or for the row swap."""
    if step == ROW_SWAP:
        return 2 * N - 1
    k = int(step) % (N // 2)
    return pow(3, k, 2 * N)


# ---------------------------------------------------------------- slots --
def decode(ctx: Context, m) -> np.ndarray:
    """Plaintext polynomial mod t -> N slot values in [0, t)."""
    ev = np.empty(ctx.N, np.uint64)
    lib().or_eval_odd(_u64(m), ev, ctx.N, ctx.t, ctx.zeta)
    return ev[ctx.slot_eval_index].astype(np.int64)


def encode(ctx: Context, slots) -> np.ndarray:
    """N slot values (any integers) -> plaintext polynomial coefficients in [0, t)."""
    v = np.mod(np.asarray(slots, dtype=np.int64), ctx.t).astype(np.uint64)
    ev = np.empty(ctx.N, np.uint64)
    ev[ctx.slot_eval_index] = v
    out = np.empty(ctx.N, np.uint64)
    lib().or_interp_odd(ev, out, ctx.N, ctx.t, ctx.zeta)
    return out


# ------------------------------------------------------------------ keys --
class SecretKey:
    def __init__(self, s: np.ndarray):
        self.s = s  # int64 ternary coefficients


class KeySwitchKey:
    """b[d][j], a[d][j]: digit d, modulus j < L+K (index L+k is p_k)."""

    def __init__(self, b: np.ndarray, a: np.ndarray, g: int):
        self.b, self.a, self.g = b, a, g


class Keys:
    def __init__(self, sk: SecretKey, pk0, pk1, rlk: Optional[KeySwitchKey],
                 galois: Dict[int, KeySwitchKey]):
        self.sk, self.pk0, self.pk1, self.rlk, self.galois = sk, pk0, pk1, rlk, galois


def secret_key(ctx: Context, seed: int) -> SecretKey:
    return SecretKey(sample_ternary(seed, DOM_SK, 0, ctx.N))


def public_key(ctx: Context, seed: int, sk: SecretKey):
    e = sample_cbd(seed, DOM_PK_E, 0, ctx.N)
    a = np.stack([sample_uniform(seed, DOM_PK_A, 0, j, ctx.N, qj) for j, qj in enumerate(ctx.q)])
    s_l = ctx.small_to_limbs(sk.s)
    e_l = ctx.small_to_limbs(e)
    prods = poly_mul_many([(a[j], s_l[j], qj) for j, qj in enumerate(ctx.q)])
    pk0 = np.stack([(qj - (prods[j] + e_l[j]) % qj) % qj for j, qj in enumerate(ctx.q)]).astype(np.uint64)
    return pk0, a


def keyswitch_key(ctx: Context, seed: int, sk: SecretKey, s_target_limbs, key_id: int) -> KeySwitchKey:
    """Key switching s_target -> s.  s_target_limbs: [L+K][N] residues of s'
    (over q_0..q_{L-1}, p_0..p_{K-1}).  key_id = 0 for relinearisation, else
    the Galois element; the ChaCha20 object id of digit d is (key_id << 8) | d."""
    N, M, dn = ctx.N, len(ctx.moduli), len(ctx.digits)
    s_l = ctx.small_to_limbs(sk.s, ctx.moduli)
    b = np.empty((dn, M, N), np.uint64)
    a = np.empty((dn, M, N), np.uint64)
    pairs = []
    for d in range(dn):
        obj = (key_id << 8) | d
        for j, m in enumerate(ctx.moduli):
            a[d, j] = sample_uniform(seed, DOM_KSK_A, obj, j, N, m)
            pairs.append((a[d, j], s_l[j], m))
    prods = poly_mul_many(pairs)
    for d in range(dn):
        obj = (key_id << 8) | d
        e_l = ctx.small_to_limbs(sample_cbd(seed, DOM_KSK_E, obj, N), ctx.moduli)
        for j, m in enumerate(ctx.moduli):
            v = (m - prods[d * M + j]) % m
            v = (v + e_l[j]) % m
            if j in ctx.digits[d]:
                v = (v + (ctx.P % m) * s_target_limbs[j] % m) % m
            b[d, j] = v
    return KeySwitchKey(b, a, key_id)


def keygen(ctx: Context, seed: int, galois_elts: Sequence[int] = (), relin: bool = True) -> Keys:
    sk = secret_key(ctx, seed)
    pk0, pk1 = public_key(ctx, seed, sk)
    s_l = ctx.small_to_limbs(sk.s, ctx.moduli)
    rlk = None
    if relin:
        s2 = np.stack(poly_mul_many([(s_l[j], s_l[j], m) for j, m in enumerate(ctx.moduli)]))
        rlk = keyswitch_key(ctx, seed, sk, s2, 0)
    gk = {}
    for g in galois_elts:
        sg = np.stack([automorph(s_l[j], m, g) for j, m in enumerate(ctx.moduli)])
        gk[int(g)] = keyswitch_key(ctx, seed, sk, sg, int(g))
    return Keys(sk, pk0, pk1, rlk, gk)


# ------------------------------------------------------- encrypt/decrypt --
def encrypt(ctx: Context, keys: Keys, m, seed: int, nonce: int) -> List[np.ndarray]:
    """m: N coefficients in [0, t).  Returns [c0, c1], each [L][N]."""
    N = ctx.N
    u = ctx.small_to_limbs(sample_ternary(seed, DOM_ENC_U, nonce, N))
    e1 = ctx.small_to_limbs(sample_cbd(seed, DOM_ENC_E1, nonce, N))
    e2 = ctx.small_to_limbs(sample_cbd(seed, DOM_ENC_E2, nonce, N))
    m = np.asarray(m, dtype=np.uint64)
    prods = poly_mul_many([(keys.pk0[j], u[j], qj) for j, qj in enumerate(ctx.q)] +
                          [(keys.pk1[j], u[j], qj) for j, qj in enumerate(ctx.q)])
    c0 = np.empty((ctx.L, N), np.uint64)
    c1 = np.empty((ctx.L, N), np.uint64)
    for j, qj in enumerate(ctx.q):
        dm = (ctx.delta % qj) * (m % qj) % qj
        c0[j] = (prods[j] + e1[j] + dm) % qj
        c1[j] = (prods[ctx.L + j] + e2[j]) % qj
    return [c0, c1]


def _phase(ctx: Context, sk: SecretKey, ct) -> np.ndarray:
    """x = c0 + c1 s (+ c2 s^2) mod Q, per limb."""
    s_l = ctx.small_to_limbs(sk.s)
    pairs = [(ct[1][j], s_l[j], qj) for j, qj in enumerate(ctx.q)]
    if len(ct) == 3:
        s2 = poly_mul_many([(s_l[j], s_l[j], qj) for j, qj in enumerate(ctx.q)])
        pairs += [(ct[2][j], s2[j], qj) for j, qj in enumerate(ctx.q)]
    prods = poly_mul_many(pairs)
    x = np.empty((ctx.L, ctx.N), np.uint64)
    for j, qj in enumerate(ctx.q):
        v = (ct[0][j] + prods[j]) % qj
        if len(ct) == 3:
            v = (v + prods[ctx.L + j]) % qj
        x[j] = v
    return x


def decrypt(ctx: Context, keys_or_sk, ct) -> np.ndarray:
    """Returns the plaintext polynomial, coefficients in [0, t)."""
    sk = keys_or_sk.sk if isinstance(keys_or_sk, Keys) else keys_or_sk
    x = ctx.crt_lift(_phase(ctx, sk, ct))
    # round(t x / Q) = floor((2 t x + Q) / (2 Q)); no ties (Q odd, gcd(t, Q) = 1).
    m = ((2 * ctx.t * x + ctx.Q) // (2 * ctx.Q)) % ctx.t
    return np.array([int(v) for v in m], dtype=np.uint64)


def noise_budget(ctx: Context, keys_or_sk, ct) -> float:
    """log2(Q) - log2(max_k |[t x_k]_Q|) - 1, in bits.  Values below 1 bit
    mean the noise has reached the decryption limit."""
    sk = keys_or_sk.sk if isinstance(keys_or_sk, Keys) else keys_or_sk
    x = ctx.crt_lift(_phase(ctx, sk, ct))
    v = (ctx.t * x) % ctx.Q
    v = np.where(v > ctx.Q // 2, ctx.Q - v, v)
    mx = max(int(z) for z in v)
    if mx == 0:
        return float(math.log2(ctx.Q) - 1)
    return float(math.log2(ctx.Q) - math.log2(mx) - 1)


# --------------------------------------------------------- homomorphic ops --
def add(ctx: Context, a, b) -> List[np.ndarray]:
    n = max(len(a), len(b))
    out = []
    for k in range(n):
        if k < len(a) and k < len(b):
            out.append(np.stack([(a[k][j] + b[k][j]) % qj for j, qj in enumerate(ctx.q)]))
        else:
            out.append((a[k] if k < len(a) else b[k]).copy())
    return out


def add_plain(ctx: Context, ct, m) -> List[np.ndarray]:
    """(c0 + Delta m, c1): m coefficients in [0, t)."""
    m = np.asarray(m, dtype=np.uint64)
    c0 = np.stack([(ct[0][j] + (ctx.delta % qj) * (m % qj) % qj) % qj for j, qj in enumerate(ctx.q)])
    return [c0] + [c.copy() for c in ct[1:]]


def centred_plain(ctx: Context, m) -> np.ndarray:
    """[m]_t: centred representatives of plaintext coefficients."""
    m = np.asarray(m, dtype=np.int64) % ctx.t
    return np.where(m > ctx.t // 2, m - ctx.t, m)


def mul_plain(ctx: Context, ct, m) -> List[np.ndarray]:
    """Each component times the centred lift of the plaintext polynomial m."""
    mt = ctx.small_to_limbs(centred_plain(ctx, m))
    pairs = [(c[j], mt[j], qj) for c in ct for j, qj in enumerate(ctx.q)]
    prods = poly_mul_many(pairs)
    return [np.stack(prods[k * ctx.L:(k + 1) * ctx.L]) for k in range(len(ct))]


def mul_scalar(ctx: Context, ct, w: int) -> List[np.ndarray]:
    """Each component times [w]_t."""
    w = int(w) % ctx.t
    if w > ctx.t // 2:
        w -= ctx.t
    return [np.stack([(c[j] * np.uint64(w % qj)) % qj for j, qj in enumerate(ctx.q)]) for c in ct]


def _aux_primes(N: int, bits_needed: int) -> List[int]:
    """Primes p = 1 mod 2N just below 2^62, enough that their product has more
    than bits_needed bits."""
    out, prod = [], 1
    k = ((1 << 62) - 1) // (2 * N)
    while prod.bit_length() <= bits_needed:
        p = k * 2 * N + 1
        k -= 1
        if _is_prime(p):
            out.append(p)
            prod *= p
    return out


def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def exact_tensor(ctx: Context, A0, A1, B0, B1):
    """Negacyclic products over Z of integer polynomials (object arrays):
    d0 = A0 B0, d1 = A0 B1 + A1 B0, d2 = A1 B1, computed modulo enough
    auxiliary primes that the centred CRT lift is the exact integer."""
    N = ctx.N
    bound = max(max(abs(int(v)) for v in X) for X in (A0, A1, B0, B1))
    bits = (2 * N * bound * bound).bit_length() + 2
    primes = _aux_primes(N, bits)
    M = math.prod(primes)
    res = []
    for p in primes:
        a0 = np.array([int(v) % p for v in A0], np.uint64)
        a1 = np.array([int(v) % p for v in A1], np.uint64)
        b0 = np.array([int(v) % p for v in B0], np.uint64)
        b1 = np.array([int(v) % p for v in B1], np.uint64)
        res.append(poly_mul_many([(a0, b0, p), (a0, b1, p), (a1, b0, p), (a1, b1, p)]))
    crt = [(M // p) * pow(M // p, -1, p) for p in primes]
    outs = []
    for kind in range(3):
        acc = np.zeros(N, dtype=object)
        for pi, p in enumerate(primes):
            r = res[pi]
            if kind == 0:
                v = r[0]
            elif kind == 1:
                v = (r[1].astype(object) + r[2].astype(object)) % p
            else:
                v = r[3]
            acc = acc + np.asarray(v).astype(object) * crt[pi]
        acc = acc % M
        acc = np.where(acc > M // 2, acc - M, acc)
        outs.append(acc)
    return outs


def mul(ctx: Context, a, b) -> List[np.ndarray]:
    """ct x ct: (|round(t d_j / Q)|_Q)_{j=0,1,2} with d the exact tensor of the
    centred lifts."""
    assert len(a) == 2 and len(b) == 2
    A0, A1 = ctx.centred_lift(a[0]), ctx.centred_lift(a[1])
    B0, B1 = ctx.centred_lift(b[0]), ctx.centred_lift(b[1])
    d = exact_tensor(ctx, A0, A1, B0, B1)
    out = []
    for dj in d:
        r = (2 * ctx.t * dj + ctx.Q) // (2 * ctx.Q)   # round(t d / Q), floor division
        out.append(ctx.reduce_int(r))
    return out


def _crt_digit(ctx: Context, x, primes) -> np.ndarray:
    """The integer in [0, Q_d) congruent to x mod each prime of the digit
    (Q_d their product), by the CRT sum; one prime: x itself."""
    if len(primes) == 1:
        return np.asarray(x[primes[0]], np.uint64)
    Qd = math.prod(ctx.q[k] for k in primes)
    acc = np.zeros(ctx.N, dtype=object)
    for k in primes:
        c = (Qd // ctx.q[k]) * pow(Qd // ctx.q[k], -1, ctx.q[k])
        acc = acc + np.asarray(x[k], np.uint64).astype(object) * c
    return acc % Qd


def _residues(v, m: int) -> np.ndarray:
    if v.dtype == object:
        return (v % m).astype(np.uint64)
    return v % np.uint64(m)


def keyswitch(ctx: Context, x, ksk: KeySwitchKey, digit_galois: int = 1):
    """x: [L][N] residues of a polynomial under s'.  Returns (k0, k1) with
    k0 + k1 s ~ x s' (mod Q).

    digit_galois = g > 1: the digits are sigma_g(|x|_{Q_d}), the automorphism
    applied to each digit as an integer polynomial (coefficients in
    (-Q_d, Q_d)), i.e. to its residues mod every modulus; then the call
    switches sigma_g(x) (each digit is still congruent to sigma_g(x) mod
    Q_d), and all rotations of one x share the digits |x|_{Q_d} -- the
    hoisted rotation."""
    L, N, K = ctx.L, ctx.N, ctx.K
    D = [_crt_digit(ctx, x, dg) for dg in ctx.digits]     # digits in [0, Q_d)
    pairs = []
    for j, m in enumerate(ctx.moduli):
        for d in range(len(D)):
            Ddj = _residues(D[d], m)
            if digit_galois != 1:
                Ddj = automorph(Ddj, m, digit_galois)
            pairs.append((Ddj, ksk.b[d, j], m))
            pairs.append((Ddj, ksk.a[d, j], m))
    prods = poly_mul_many(pairs)
    nd = len(D)
    u0 = np.empty((L + K, N), np.uint64)
    u1 = np.empty((L + K, N), np.uint64)
    for j, m in enumerate(ctx.moduli):
        s0 = np.zeros(N, dtype=np.uint64)
        s1 = np.zeros(N, dtype=np.uint64)
        for d in range(nd):
            s0 = (s0 + prods[(j * nd + d) * 2]) % m
            s1 = (s1 + prods[(j * nd + d) * 2 + 1]) % m
        u0[j], u1[j] = s0, s1
    P = ctx.P
    out = []
    for u in (u0, u1):
        # [u mod P]_P, centred: the CRT lift over the special primes
        if K == 1:
            uP = u[L].astype(np.int64)
        else:
            uP = np.zeros(N, dtype=object)
            for k, pk in enumerate(ctx.special):
                uP = uP + u[L + k].astype(object) * ((P // pk) * pow(P // pk, -1, pk))
            uP = uP % P
        uPc = np.where(uP > P // 2, uP - P, uP)
        limbs = np.empty((L, N), np.uint64)
        for j, qj in enumerate(ctx.q):
            pinv = pow(P, -1, qj)
            r = (uPc % qj).astype(np.int64)
            diff = (u[j].astype(np.int64) - r) % qj
            limbs[j] = (diff.astype(np.uint64) * np.uint64(pinv)) % np.uint64(qj)
        out.append(limbs)
    return out[0], out[1]


def relin(ctx: Context, ct3, rlk: KeySwitchKey) -> List[np.ndarray]:
    k0, k1 = keyswitch(ctx, ct3[2], rlk)
    return [np.stack([(ct3[0][j] + k0[j]) % qj for j, qj in enumerate(ctx.q)]),
            np.stack([(ct3[1][j] + k1[j]) % qj for j, qj in enumerate(ctx.q)])]


def apply_galois(ctx: Context, ct, g: int) -> List[np.ndarray]:
    return [np.stack([automorph(c[j], qj, g) for j, qj in enumerate(ctx.q)]) for c in ct]


def rotate(ctx: Context, ct, step, keys: Keys) -> List[np.ndarray]:
    """rotate(+k): left rotation of each slot row by k; ROW_SWAP swaps rows."""
    g = galois_element(ctx.N, step)
    if g == 1:
        return [c.copy() for c in ct]
    ksk = keys.galois[g]
    c0g, c1g = apply_galois(ctx, ct, g)
    k0, k1 = keyswitch(ctx, c1g, ksk)
    return [np.stack([(c0g[j] + k0[j]) % qj for j, qj in enumerate(ctx.q)]), k1]


def rotate_hoisted(ctx: Context, ct, step, keys: Keys) -> List[np.ndarray]:
    """The same rotation as `rotate` (it decrypts to the same slots), with the
    key switch's digits taken before the automorphism: digit d is
    sigma_g(|c1|_{Q_d}) (see keyswitch).  Rotations of one ciphertext by
    several g then share |c1|_{Q_d} and its reductions to every modulus; the
    words differ from `rotate`'s where sigma_g negates a coefficient."""
    g = galois_element(ctx.N, step)
    if g == 1:
        return [c.copy() for c in ct]
    ksk = keys.galois[g]
    c0g = [automorph(ct[0][j], qj, g) for j, qj in enumerate(ctx.q)]
    k0, k1 = keyswitch(ctx, ct[1], ksk, digit_galois=g)
    return [np.stack([(c0g[j] + k0[j]) % qj for j, qj in enumerate(ctx.q)]), k1]


def square(ctx: Context, ct, keys: Keys) -> List[np.ndarray]:
    return relin(ctx, mul(ctx, ct, ct), keys.rlk)
