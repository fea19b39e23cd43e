/*
 * Reference (oracle) polynomial arithmetic for BFV over R_m = Z_m[X]/(X^N+1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file, and everything else under oracle/, is
 * the slow, plainly written CPU reference that the GPU library is checked
 * against.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does.  It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * The paper (Sec. 3.1, "Homomorphic Encryption", and App. A "Rings") fixes the
 * ring: polynomials with coefficients mod m, reduced modulo X^N + 1 with N a
 * power of two.  Everything here is a plain definition of an operation on that
 * ring:
 *   - or_poly_mul_schoolbook: the negacyclic product by its definition,
 *       c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j   (mod m)
 *   - or_poly_mul: the same product through a textbook psi-twisted
 *       number-theoretic transform (a library-style primitive, checked against
 *       the schoolbook product by the tests);
 *   - or_eval_odd / or_interp_odd: evaluation of a polynomial at all odd powers
 *       of a primitive 2N-th root, and its inverse (used for slot encoding,
 *       Sec. 3.1: with a 2N-th root of unity mod p the ring splits into N slots);
 *   - or_automorph: a(X) -> a(X^g) for odd g (the rotations of Sec. 3.1 are
 *       such automorphisms on the slot vector);
 *   - ChaCha20 block function (RFC 8439, Sec. 2.3) and the three samplers
 *       built on it (uniform mod m, ternary, centred binomial).
 * Moduli are odd primes below 2^62; products use unsigned __int128 (plain
 * 64-bit products for moduli below 2^32).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
    if (m <= 0xFFFFFFFFull) return (a * b) % m; /* a, b < m: product < 2^64 */
    return (uint64_t)(((u128)a * b) % m);
}
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t m) {
    uint64_t s = a + b;
    return s >= m ? s - m : s;
}
static uint64_t submod(uint64_t a, uint64_t b, uint64_t m) {
    return a >= b ? a - b : a + m - b;
}
static uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    b %= m;
    while (e) {
        if (e & 1) r = mulmod(r, b, m);
        b = mulmod(b, b, m);
        e >>= 1;
    }
    return r;
}
static uint64_t invmod(uint64_t a, uint64_t m) { /* m prime */
    return powmod(a, m - 2, m);
}

/* Smallest g in [2, m) with g^N == -1 (mod m); such a g has order exactly 2N
 * because 2N is a power of two.  Returns 0 if none exists (m != 1 mod 2N). */
uint64_t or_min_root_2n(uint64_t m, uint32_t N) {
    if ((m - 1) % (2ull * N) != 0) return 0;
    for (uint64_t g = 2; g < m; ++g)
        if (powmod(g, N, m) == m - 1) return g;
    return 0;
}

/* Any primitive 2N-th root (fast: x^((m-1)/2N) for increasing x). */
static uint64_t some_root_2n(uint64_t m, uint32_t N) {
    uint64_t e = (m - 1) / (2ull * N);
    for (uint64_t x = 2; x < m; ++x) {
        uint64_t r = powmod(x, e, m);
        if (powmod(r, N, m) == m - 1) return r;
    }
    return 0;
}

/* In-place cyclic DFT of length N over Z_m with root w (w^N = 1), natural
 * order in and out: out_k = sum_j a_j w^{jk}.  Iterative radix-2 with an
 * explicit bit-reversal permutation. */
static void cyclic_dft(uint64_t *a, uint32_t N, uint64_t w, uint64_t m) {
    uint32_t logn = 0;
    while ((1u << logn) < N) ++logn;
    for (uint32_t i = 0; i < N; ++i) {
        uint32_t r = 0;
        for (uint32_t b = 0; b < logn; ++b)
            if (i & (1u << b)) r |= 1u << (logn - 1 - b);
        if (r > i) { uint64_t t = a[i]; a[i] = a[r]; a[r] = t; }
    }
    /* pw[j] = w^j for j < N/2; a stage of length len uses w^(N/len). */
    uint64_t *pw = (uint64_t *)malloc(sizeof(uint64_t) * (N / 2 + 1));
    pw[0] = 1 % m;
    for (uint32_t j = 1; j < N / 2; ++j) pw[j] = mulmod(pw[j - 1], w, m);
    for (uint32_t len = 2; len <= N; len <<= 1) {
        uint32_t step = N / len;
        for (uint32_t s = 0; s < N; s += len) {
            for (uint32_t j = 0; j < len / 2; ++j) {
                uint64_t u = a[s + j];
                uint64_t v = mulmod(a[s + j + len / 2], pw[j * step], m);
                a[s + j] = addmod(u, v, m);
                a[s + j + len / 2] = submod(u, v, m);
            }
        }
    }
    free(pw);
}

/* out[k] = a(root^(2k+1)) for k = 0..N-1 (root a primitive 2N-th root).
 * Written as: twist a_j by root^j, then a cyclic DFT with root^2. */
void or_eval_odd(const uint64_t *a, uint64_t *out, uint32_t N, uint64_t m, uint64_t root) {
    uint64_t x = 1;
    for (uint32_t j = 0; j < N; ++j) {
        out[j] = mulmod(a[j] % m, x, m);
        x = mulmod(x, root, m);
    }
    cyclic_dft(out, N, mulmod(root, root, m), m);
}

/* Inverse of or_eval_odd: given v[k] = a(root^(2k+1)), recover a. */
void or_interp_odd(const uint64_t *v, uint64_t *a, uint32_t N, uint64_t m, uint64_t root) {
    for (uint32_t j = 0; j < N; ++j) a[j] = v[j] % m;
    uint64_t rinv = invmod(root, m);
    cyclic_dft(a, N, mulmod(rinv, rinv, m), m);
    uint64_t ninv = invmod(N % m, m);
    uint64_t x = ninv;
    for (uint32_t j = 0; j < N; ++j) {
        a[j] = mulmod(a[j], x, m);
        x = mulmod(x, rinv, m);
    }
}

/* Negacyclic product by definition, O(N^2). */
void or_poly_mul_schoolbook(const uint64_t *a, const uint64_t *b, uint64_t *out,
                            uint32_t N, uint64_t m) {
    for (uint32_t k = 0; k < N; ++k) out[k] = 0;
    for (uint32_t i = 0; i < N; ++i) {
        uint64_t ai = a[i] % m;
        if (!ai) continue;
        for (uint32_t j = 0; j < N; ++j) {
            uint64_t p = mulmod(ai, b[j] % m, m);
            uint32_t k = i + j;
            if (k < N) out[k] = addmod(out[k], p, m);
            else out[k - N] = submod(out[k - N], p, m);
        }
    }
}

/* Negacyclic product via evaluation at the odd powers of a 2N-th root:
 * a*b mod (X^N+1) is the unique polynomial whose values at the roots of
 * X^N+1 are the products of the values of a and b. */
void or_poly_mul(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t N, uint64_t m) {
    uint64_t root = some_root_2n(m, N);
    uint64_t *fa = (uint64_t *)malloc(sizeof(uint64_t) * N);
    uint64_t *fb = (uint64_t *)malloc(sizeof(uint64_t) * N);
    or_eval_odd(a, fa, N, m, root);
    or_eval_odd(b, fb, N, m, root);
    for (uint32_t k = 0; k < N; ++k) fa[k] = mulmod(fa[k], fb[k], m);
    or_interp_odd(fa, out, N, m, root);
    free(fa);
    free(fb);
}

/* Batched negacyclic products: out[i] = a[i] * b[i] (mod m[i]) for i < count,
 * each polynomial N coefficients, contiguous.  Convenience for the Python
 * side; each product is an independent call of or_poly_mul, so they may run
 * on several host threads. */
void or_poly_mul_many(const uint64_t *a, const uint64_t *b, uint64_t *out, uint32_t N,
                      const uint64_t *m, uint32_t count) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < (int64_t)count; ++i)
        or_poly_mul(a + (size_t)i * N, b + (size_t)i * N, out + (size_t)i * N, N, m[i]);
}

/* sigma_g: a(X) -> a(X^g), g odd.  X^{i g} = X^{(i g mod 2N)}, and
 * X^{N + r} = -X^r in R. */
void or_automorph(const uint64_t *a, uint64_t *out, uint32_t N, uint64_t m, uint64_t g) {
    uint64_t twoN = 2ull * N;
    for (uint32_t i = 0; i < N; ++i) {
        uint64_t e = ((uint64_t)i * (g % twoN)) % twoN;
        uint64_t v = a[i] % m;
        if (e < N) out[e] = v;
        else out[e - N] = v ? m - v : 0;
    }
}

/* ---------------- ChaCha20 (RFC 8439, Sec. 2.1-2.3) ---------------- */
static uint32_t rotl32(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }
#define QR(a, b, c, d)                      \
    do {                                    \
        a += b; d ^= a; d = rotl32(d, 16);  \
        c += d; b ^= c; b = rotl32(b, 12);  \
        a += b; d ^= a; d = rotl32(d, 8);   \
        c += d; b ^= c; b = rotl32(b, 7);   \
    } while (0)

void or_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3],
                       uint32_t out[16]) {
    uint32_t s[16];
    s[0] = 0x61707865u; s[1] = 0x3320646eu; s[2] = 0x79622d32u; s[3] = 0x6b206574u;
    for (int i = 0; i < 8; ++i) s[4 + i] = key[i];
    s[12] = counter;
    s[13] = nonce[0]; s[14] = nonce[1]; s[15] = nonce[2];
    uint32_t x[16];
    memcpy(x, s, sizeof x);
    for (int r = 0; r < 10; ++r) {
        QR(x[0], x[4], x[8], x[12]);
        QR(x[1], x[5], x[9], x[13]);
        QR(x[2], x[6], x[10], x[14]);
        QR(x[3], x[7], x[11], x[15]);
        QR(x[0], x[5], x[10], x[15]);
        QR(x[1], x[6], x[11], x[12]);
        QR(x[2], x[7], x[8], x[13]);
        QR(x[3], x[4], x[9], x[14]);
    }
    for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

/* The random word of coefficient i for stream (key, domain, object, limb):
 * key = the eight 32-bit words of the 256-bit seed, least significant first
 * (a seed below 2^64 leaves words 2..7 zero), nonce = (domain, object, limb),
 * block counter = i / 8, word = 64-bit little-endian word (i mod 8) of the
 * 64-byte block. */
void or_stream_words(const uint32_t *key, uint32_t domain, uint32_t object, uint32_t limb,
                     uint32_t n, uint64_t *out) {
    uint32_t nonce[3] = {domain, object, limb};
    uint32_t blk[16];
    for (uint32_t i = 0; i < n; ++i) {
        if (i % 8 == 0) or_chacha20_block(key, i / 8, nonce, blk);
        uint32_t w = i % 8;
        out[i] = (uint64_t)blk[2 * w] | ((uint64_t)blk[2 * w + 1] << 32);
    }
}

/* Uniform residue mod m: word mod m. */
void or_sample_uniform(const uint32_t *key, uint32_t domain, uint32_t object, uint32_t limb,
                       uint32_t n, uint64_t m, uint64_t *out) {
    or_stream_words(key, domain, object, limb, n, out);
    for (uint32_t i = 0; i < n; ++i) out[i] %= m;
}

/* Ternary value in {-1,0,1}: (word mod 3) - 1. */
void or_sample_ternary(const uint32_t *key, uint32_t domain, uint32_t object, uint32_t n,
                       int64_t *out) {
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * n);
    or_stream_words(key, domain, object, 0, n, w);
    for (uint32_t i = 0; i < n; ++i) out[i] = (int64_t)(w[i] % 3) - 1;
    free(w);
}

/* Centred binomial with 21 coin pairs: popcount of the low 21 bits minus the
 * popcount of the next 21 bits (variance 10.5). */
void or_sample_cbd(const uint32_t *key, uint32_t domain, uint32_t object, uint32_t n,
                   int64_t *out) {
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * n);
    or_stream_words(key, domain, object, 0, n, w);
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t lo = w[i] & 0x1FFFFFull, hi = (w[i] >> 21) & 0x1FFFFFull;
        int64_t c = 0;
        for (int b = 0; b < 21; ++b) c += (int64_t)((lo >> b) & 1) - (int64_t)((hi >> b) & 1);
        out[i] = c;
    }
    free(w);
}

/* Host threads the batched products may use (reported with CPU timings). */
#ifdef _OPENMP
#include <omp.h>
int or_max_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int or_max_threads(void) { return 1; }
void or_set_threads(int n) { (void)n; }
#endif
