"""Independent brute-force BFV in pure Python integers, for tiny N (<= 64).

Written separately from the oracle (oracle/bfv.py + oracle/bfv_ref.c) to pin
it: everything here is the plain definition, with no transforms and no
auxiliary primes:
  - negacyclic products by the double sum over i + j;
  - ciphertext products over Z of the centred lifts, then round(t d / Q) with
    exact rational arithmetic;
  - slot values by evaluating m at zeta^e with Horner's rule, and encoding by
    the inverse formula m_j = N^-1 sum_k v_k w_k^-j over the N roots w_k of
    X^N + 1;
  - ChaCha20 as RFC 8439 describes it.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List

MASK32 = 0xFFFFFFFF


# ------------------------------------------------------------- ChaCha20 --
def _rotl(x, n):
    return ((x << n) | (x >> (32 - n))) & MASK32


def quarter_round(a, b, c, d):
    a = (a + b) & MASK32; d = _rotl(d ^ a, 16)
    c = (c + d) & MASK32; b = _rotl(b ^ c, 12)
    a = (a + b) & MASK32; d = _rotl(d ^ a, 8)
    c = (c + d) & MASK32; b = _rotl(b ^ c, 7)
    return a, b, c, d


def chacha20_block(key: List[int], counter: int, nonce: List[int]) -> List[int]:
    init = [0x61707865, 0x3320646E, 0x79622D32, 0x6B206574] + list(key) + [counter] + list(nonce)
    x = list(init)
    for _ in range(10):
        for (i, j, k, l) in ((0, 4, 8, 12), (1, 5, 9, 13), (2, 6, 10, 14), (3, 7, 11, 15),
                             (0, 5, 10, 15), (1, 6, 11, 12), (2, 7, 8, 13), (3, 4, 9, 14)):
            x[i], x[j], x[k], x[l] = quarter_round(x[i], x[j], x[k], x[l])
    return [(x[i] + init[i]) & MASK32 for i in range(16)]


def words(seed, domain, obj, limb, n):
    key = [(seed >> (32 * k)) & MASK32 for k in range(8)]   # the 256-bit seed, low word first
    out = []
    for i in range(n):
        blk = chacha20_block(key, i // 8, [domain, obj, limb])
        w = i % 8
        out.append(blk[2 * w] | (blk[2 * w + 1] << 32))
    return out


def uniform(seed, dom, obj, limb, n, m):
    return [w % m for w in words(seed, dom, obj, limb, n)]


def ternary(seed, dom, obj, n):
    return [w % 3 - 1 for w in words(seed, dom, obj, 0, n)]


def cbd(seed, dom, obj, n):
    out = []
    for w in words(seed, dom, obj, 0, n):
        lo, hi = w & 0x1FFFFF, (w >> 21) & 0x1FFFFF
        out.append(bin(lo).count("1") - bin(hi).count("1"))
    return out


# ---------------------------------------------------------------- ring --
def negacyclic(a, b, m=None):
    N = len(a)
    c = [0] * N
    for i in range(N):
        for j in range(N):
            if i + j < N:
                c[i + j] += a[i] * b[j]
            else:
                c[i + j - N] -= a[i] * b[j]
    return c if m is None else [x % m for x in c]


def automorphism(a, g):
    N = len(a)
    out = [0] * N
    for i, v in enumerate(a):
        e = (i * g) % (2 * N)
        if e < N:
            out[e] += v
        else:
            out[e - N] -= v
    return out


class Tiny:
    """special: the special prime P, or a tuple of K special primes; key
    switching then takes digits of K consecutive ciphertext primes."""

    def __init__(self, N, t, q, special):
        self.special = list(special) if isinstance(special, (tuple, list)) else [special]
        self.N, self.t, self.q = N, t, list(q)
        self.P = 1
        for p in self.special:
            self.P *= p
        self.L = len(q)
        self.Q = 1
        for x in q:
            self.Q *= x
        self.delta = self.Q // t
        self.moduli = self.q + self.special
        K = len(self.special)
        self.groups = [list(range(i, min(i + K, self.L))) for i in range(0, self.L, K)]
        self.zeta = next(g for g in range(2, t) if pow(g, N, t) == t - 1)

    # slots
    def slot_exp(self, s):
        n2 = self.N // 2
        r, i = divmod(s, n2)
        return (pow(2 * self.N - 1, r, 2 * self.N) * pow(3, i, 2 * self.N)) % (2 * self.N)

    def decode(self, m):
        out = []
        for s in range(self.N):
            x = pow(self.zeta, self.slot_exp(s), self.t)
            acc = 0
            for c in reversed(m):
                acc = (acc * x + c) % self.t
            out.append(acc)
        return out

    def encode(self, v):
        N, t = self.N, self.t
        ninv = pow(N, -1, t)
        pts = [(pow(self.zeta, self.slot_exp(s), t), v[s] % t) for s in range(N)]
        return [ninv * sum(val * pow(w, -j, t) for w, val in pts) % t for j in range(N)]

    # integer <-> limbs
    def limbs(self, poly, moduli=None):
        moduli = self.q if moduli is None else moduli
        return [[c % m for c in poly] for m in moduli]

    def lift(self, limbs):
        out = []
        for k in range(self.N):
            x = 0
            for i, qi in enumerate(self.q):
                Qi = self.Q // qi
                x += limbs[i][k] * Qi * pow(Qi, -1, qi)
            out.append(x % self.Q)
        return out

    def centred(self, limbs):
        return [x - self.Q if x > self.Q // 2 else x for x in self.lift(limbs)]

    # keys
    def keygen(self, seed, galois):
        N, L = self.N, self.L
        s = ternary(seed, 1, 0, N)
        e = cbd(seed, 3, 0, N)
        a = [uniform(seed, 2, 0, j, N, qj) for j, qj in enumerate(self.q)]
        pk0 = [[(-(x + y)) % qj for x, y in zip(negacyclic(a[j], s, qj), e)]
               for j, qj in enumerate(self.q)]
        keys = {"s": s, "pk0": pk0, "pk1": a}
        keys["rlk"] = self.ksk(seed, s, negacyclic(s, s), 0)
        keys["gal"] = {g: self.ksk(seed, s, automorphism(s, g), g) for g in galois}
        return keys

    def ksk(self, seed, s, s_target, key_id):
        N, M = self.N, len(self.moduli)
        b = [[None] * M for _ in self.groups]
        a = [[None] * M for _ in self.groups]
        for i, grp in enumerate(self.groups):
            obj = (key_id << 8) | i
            e = cbd(seed, 5, obj, N)
            for j, m in enumerate(self.moduli):
                aij = uniform(seed, 4, obj, j, N, m)
                as_ = negacyclic(aij, s, m)
                v = [(-x + y) % m for x, y in zip(as_, e)]
                if j in grp:
                    v = [(x + (self.P % m) * st) % m for x, st in zip(v, s_target)]
                a[i][j], b[i][j] = aij, v
        return (b, a)

    @staticmethod
    def garner(res, mods):
        """The integer in [0, prod mods) with the given residues, built one
        modulus at a time: v <- v + (prod so far) * ((r - v) / (prod so far)
        mod m)."""
        v, w = 0, 1
        for r, m in zip(res, mods):
            v += w * (((r - v) * pow(w, -1, m)) % m)
            w *= m
        return v

    def encrypt(self, keys, m, seed, nonce):
        N = self.N
        u = ternary(seed, 6, nonce, N)
        e1 = cbd(seed, 7, nonce, N)
        e2 = cbd(seed, 8, nonce, N)
        c0, c1 = [], []
        for j, qj in enumerate(self.q):
            p0 = negacyclic(keys["pk0"][j], u, qj)
            p1 = negacyclic(keys["pk1"][j], u, qj)
            c0.append([(x + y + self.delta * mm) % qj for x, y, mm in zip(p0, e1, m)])
            c1.append([(x + y) % qj for x, y in zip(p1, e2)])
        return [c0, c1]

    def decrypt(self, keys, ct):
        s = keys["s"]
        x = [0] * self.N
        spow = [1] + [0] * (self.N - 1)
        for comp in ct:
            cz = self.lift(comp)
            term = negacyclic(cz, spow)
            x = [(a + b) % self.Q for a, b in zip(x, term)]
            spow = negacyclic(spow, s)
        out = []
        for v in x:
            r = Fraction(self.t * v, self.Q)
            out.append(int((r + Fraction(1, 2)) // 1) % self.t)
        return out

    # operations (coefficient form, limbs)
    def add(self, a, b):
        return [[[(x + y) % qj for x, y in zip(a[k][j], b[k][j])] for j, qj in enumerate(self.q)]
                for k in range(len(a))]

    def add_plain(self, ct, m):
        c0 = [[(x + self.delta * mm) % qj for x, mm in zip(ct[0][j], m)] for j, qj in enumerate(self.q)]
        return [c0] + ct[1:]

    def mul_plain(self, ct, m):
        mc = [x - self.t if x > self.t // 2 else x for x in (v % self.t for v in m)]
        return [[negacyclic(c[j], mc, qj) for j, qj in enumerate(self.q)] for c in ct]

    def mul_scalar(self, ct, w):
        w %= self.t
        if w > self.t // 2:
            w -= self.t
        return [[[(x * w) % qj for x in c[j]] for j, qj in enumerate(self.q)] for c in ct]

    def mul(self, a, b):
        A0, A1 = self.centred(a[0]), self.centred(a[1])
        B0, B1 = self.centred(b[0]), self.centred(b[1])
        d0 = negacyclic(A0, B0)
        d1 = [x + y for x, y in zip(negacyclic(A0, B1), negacyclic(A1, B0))]
        d2 = negacyclic(A1, B1)
        out = []
        for d in (d0, d1, d2):
            r = [int((Fraction(self.t * x, self.Q) + Fraction(1, 2)) // 1) for x in d]
            out.append(self.limbs(r))
        return out

    def keyswitch(self, x, key, digit_g=1):
        """Digit d is x mod Q_d (its primes' product) in [0, Q_d).  digit_g > 1:
        the automorphism of each digit taken as an integer polynomial (signed),
        reduced mod each modulus."""
        b, a = key
        L, N, P = self.L, self.N, self.P
        digits = [[self.garner([x[k][c] for k in grp], [self.q[k] for k in grp]) for c in range(N)]
                  for grp in self.groups]
        u0, u1 = [], []
        for j, m in enumerate(self.moduli):
            s0 = [0] * N
            s1 = [0] * N
            for i, dg in enumerate(digits):
                xi = automorphism(dg, digit_g) if digit_g != 1 else dg
                Di = [v % m for v in xi]
                s0 = [(p + r) % m for p, r in zip(s0, negacyclic(Di, b[i][j], m))]
                s1 = [(p + r) % m for p, r in zip(s1, negacyclic(Di, a[i][j], m))]
            u0.append(s0)
            u1.append(s1)
        out = []
        sp = self.special
        for u in (u0, u1):
            uP = [self.garner([u[L + k][c] for k in range(len(sp))], sp) for c in range(N)]
            uP = [v - P if v > P // 2 else v for v in uP]
            out.append([[((u[j][k] - uP[k]) * pow(P, -1, qj)) % qj for k in range(N)]
                        for j, qj in enumerate(self.q)])
        return out

    def relin(self, ct3, keys):
        k0, k1 = self.keyswitch(ct3[2], keys["rlk"])
        return self.add([ct3[0], ct3[1]], [k0, k1])

    def rotate(self, ct, g, keys):
        c0 = [[v % qj for v in automorphism(ct[0][j], g)] for j, qj in enumerate(self.q)]
        c1 = [[v % qj for v in automorphism(ct[1][j], g)] for j, qj in enumerate(self.q)]
        k0, k1 = self.keyswitch(c1, keys["gal"][g])
        return self.add([c0, k1], [k0, [[0] * self.N for _ in self.q]])

    def rotate_hoisted(self, ct, g, keys):
        """Digits from c1 before the automorphism, permuted afterwards."""
        c0 = [[v % qj for v in automorphism(ct[0][j], g)] for j, qj in enumerate(self.q)]
        k0, k1 = self.keyswitch(ct[1], keys["gal"][g], digit_g=g)
        return self.add([c0, k1], [k0, [[0] * self.N for _ in self.q]])
