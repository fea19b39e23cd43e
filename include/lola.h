/*
 * liblola: BFV ciphertext arithmetic over R_q = Z_q[X]/(X^N + 1) in RNS form on
 * one MI355X (gfx950), and the LoLa layer schedules built on it.
 *
 * The operations are the ones the paper (Brutzkus, Elisha, Gilad-Bachrach,
 * "Low Latency Privacy Preserving Inference") relies on:
 *   - Sec. 3.1 (Homomorphic Encryption): encryption E, decryption D, the
 *     homomorphic sum and product, the plaintext ring Z_p[x]/(x^n+1) viewed as
 *     n slots when p has a 2n-th root of unity, and the two rotations of the
 *     2 x n/2 slot matrix (row swap, column rotation);
 *   - Sec. 4.2.2 (Convolution vector - row major): message times scalar;
 *   - Sec. 4.2 (vector representations and matrix-vector recipes) and Sec. 4.3 /
 *     App. C (the MNIST pipeline): the layer compiler and network evaluation.
 * Key switching (relinearisation, rotation keys) and the RNS/NTT form are how
 * BFV realises those operations; the paper uses them through its library.
 *
 * Conventions for every call:
 *   - Ownership: the caller owns every buffer.  Pointers named *_dev are device
 *     memory on the context's GPU, *_host host memory.  The library never frees
 *     caller memory; it owns only lola_ctx / lola_plan and their scratch.
 *   - Asynchrony: calls enqueue work on `stream` (a hipStream_t; NULL = the
 *     default stream) and return; device faults surface at the caller's next
 *     synchronisation.  Calls that return host results (noted) synchronise.
 *   - One context must not be used from two streams at once (shared scratch).
 *   - Layouts (uint32 words, little endian):
 *       polynomial   [L][N]       one limb (residues mod q_i) per prime
 *       ciphertext   [size][L][N] size 2 (or 3 after lola_mul); device form is
 *                                 the NTT (evaluation) form described below
 *       plaintext    [N]          coefficients mod t (lola_encode output)
 *       mul-form pt  [L][N]       from lola_plain_mul_form
 *       add-form pt  [L][N]       from lola_plain_add_form
 *       secret key   [L+K][N]     NTT form mod q_0..q_{L-1} and the K special primes
 *       public key   [2][L][N]
 *       switch key   [dn][2][L+K][N]  (relinearisation or one Galois element;
 *                                 dn digits of K ciphertext primes, K = 1 or 2,
 *                                 see lola_params)
 *     Device forms are internal: NTT evaluation order with Montgomery scaling
 *     on key and mul-form data.  lola_to_coeff / lola_*_export give the
 *     canonical coefficient form (residues in [0, q_i)) used for comparisons.
 *   - Errors: 0 on success, a negative LOLA_E_* code otherwise; the message of
 *     the last error on the calling thread is lola_last_error().  Shapes are
 *     checked against the context; pointers are not dereferenced on the host.
 *   - Aliasing: element-wise calls (add, add_plain, mul_plain, mul_scalar) may
 *     run in place; lola_mul, lola_relin and lola_rotate may not alias their
 *     output with an input.
 */
#ifndef LOLA_H
#define LOLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *lola_stream; /* hipStream_t */

enum {
    LOLA_OK = 0,
    LOLA_E_INVAL = -1,       /* bad argument (null pointer, out-of-range value) */
    LOLA_E_PARAMS = -2,      /* a modulus is not prime / not 1 mod 2N / too large; gcd(t, Q) != 1 */
    LOLA_E_INSECURE = -3,    /* log2(Q P) above the 128-bit cap for N (ternary secret) */
    LOLA_E_SHAPE = -4,       /* size / count does not match the context */
    LOLA_E_NOKEY = -5,       /* a rotation needs a Galois key that was not given */
    LOLA_E_NOMEM = -6,       /* device allocation of scratch failed */
    LOLA_E_DEVICE = -7,      /* a HIP runtime call failed */
    LOLA_E_UNSUPPORTED = -8  /* layer pattern or size the compiler does not handle */
};

#define LOLA_ROW_SWAP 0x7fffffff /* step value of the row swap in rotation calls */

/* Parameter set.  N in {1024, 2048, 4096, 8192, 16384}; t prime, t = 1 mod 2N,
 * t < 2^26; q[0..L-1], P (and P2) distinct primes below 2^30, each = 1 mod
 * 2N; 1 <= L <= 12.  Unless allow_insecure, log2(Q*P) must not exceed the
 * homomorphic-encryption standard's 128-bit classical cap for N (27, 54, 109,
 * 218, 438 for N = 1024 ... 16384).
 * Key switching (hybrid, with special primes): P2 = 0 gives one special
 * prime P and one digit per ciphertext prime (L digits); P2 != 0 gives two
 * special primes P, P2 (their product is the P of the mod-down) and digits
 * of two consecutive ciphertext primes (ceil(L/2) digits: fewer transforms,
 * key products and key words per key switch at the same noise), and then
 * every modulus must exceed 2^29.  K below is the number of special primes,
 * dn the number of digits. */
typedef struct {
    uint32_t N;
    uint32_t t;
    uint32_t L;
    const uint32_t *q; /* host array of L primes */
    uint32_t P;
    int allow_insecure;
    uint32_t P2;       /* second special prime, or 0 */
} lola_params;

typedef struct lola_ctx lola_ctx;

typedef struct {
    uint32_t N, L, t, n_aux;       /* n_aux: primes of the exact product's extra basis */
    uint64_t ct_words;             /* 2*L*N */
    uint64_t poly_words;           /* L*N */
    uint64_t sk_words;             /* (L+K)*N */
    uint64_t ksk_words;            /* dn*2*(L+K)*N */
    uint64_t scratch_bytes;        /* current scratch arena */
    uint32_t K, dnum;              /* special primes, key-switching digits */
} lola_info;

/* ---------------------------------------------------------------- context */
/* Validates params (errors above), builds NTT tables for every prime, the
 * exact mixed-radix constants, and selects the auxiliary basis.  Device =
 * HIP device ordinal; the context's calls must run with that device current. */
int lola_ctx_create(const lola_params *params, int device, lola_ctx **out);
void lola_ctx_destroy(lola_ctx *ctx);
int lola_ctx_info(const lola_ctx *ctx, lola_info *info);
/* Pre-sizes the scratch arena for batches of up to n ciphertexts so later
 * calls do not allocate (e.g. before stream capture). */
int lola_reserve(lola_ctx *ctx, uint32_t n_ct);

/* Galois element of a rotation: step > 0 rotates every slot row left by step
 * (output slot (r,i) takes input slot (r, i+step)), step < 0 right, and
 * LOLA_ROW_SWAP swaps the two rows (Sec. 3.1).  Returns 3^step mod 2N or
 * 2N-1; 0 on a bad N. */
uint32_t lola_galois_element(uint32_t N, int32_t step);

/* ------------------------------------------------------------------- keys */
/* Keys of the scheme of Sec. 3.1 (the paper takes BFV from its library; the
 * public-key and switching-key forms are this library's reading: ternary s,
 * pk = (-(a s + e), a), hybrid switching keys with special primes: digit d
 * of K consecutive ciphertext primes carries P s' at exactly its own primes,
 * P the special primes' product; one digit per prime with one special
 * prime, or digits of two primes with two).  sk_dev [L+K][N], pk_dev
 * [2][L][N], ksk_dev [dn][2][L+K][N] (caller-owned device buffers, written).
 * Errors:
 * LOLA_E_INVAL (null pointer, bad Galois element).
 * Random values come from ChaCha20 (RFC 8439) with key = (seed lo, seed hi,
 * k2..k7), k2..k7 the context's key words, nonce = (domain, object, limb),
 * one 64-bit word per coefficient; uniform = word mod m, ternary = word mod 3
 * - 1, error = centred binomial popcount(w & 0x1fffff) - popcount((w >> 21)
 * & 0x1fffff).  Security: the secret key, the switching keys and every
 * encryption's randomness follow from the key, so seed and key words must be
 * secret and uniformly random; with the key words left at zero the key has
 * only the seed's 64 bits, fit for tests, not for deployment.
 * lola_set_key_words sets k2..k7 (words_host: 6 words; NULL = zeros) for
 * every later key generation and encryption on the context (a 256-bit key). */
int lola_set_key_words(lola_ctx *ctx, const uint32_t *words_host);
int lola_keygen_secret(lola_ctx *ctx, uint64_t seed, uint32_t *sk_dev, lola_stream stream);
int lola_keygen_public(lola_ctx *ctx, uint64_t seed, const uint32_t *sk_dev, uint32_t *pk_dev,
                       lola_stream stream);
/* Switching key from s^2 (galois = 0) or from sigma_galois(s) to s. */
int lola_keygen_switch(lola_ctx *ctx, uint64_t seed, const uint32_t *sk_dev, uint32_t galois,
                       uint32_t *ksk_dev, lola_stream stream);

/* ------------------------------------------------------------- plaintexts */
/* Slot encoding (Sec. 3.1 batching): slot (r, i) = r*N/2 + i of the
 * plaintext m is m(zeta^e), e = (2N-1)^r 3^i mod 2N, zeta the smallest
 * primitive 2N-th root of unity mod t.  slots_dev: N int64 (any integers,
 * reduced mod t); pt_dev: N words in [0, t). */
int lola_encode(lola_ctx *ctx, const int64_t *slots_dev, uint32_t *pt_dev, lola_stream stream);
int lola_decode(lola_ctx *ctx, const uint32_t *pt_dev, int64_t *slots_dev, lola_stream stream);
/* The same over n messages stored back to back: slots_dev n * N int64,
 * pt_dev n * N words; message i equals the single call on message i.  A
 * client's whole input (25 messages of the MNIST network) is one call. */
int lola_encode_batch(lola_ctx *ctx, const int64_t *slots_dev, uint32_t n, uint32_t *pt_dev, lola_stream stream);
int lola_decode_batch(lola_ctx *ctx, const uint32_t *pt_dev, uint32_t n, int64_t *slots_dev, lola_stream stream);
/* Plaintext forms: mul form = centred lift [m]_t per prime (for
 * lola_mul_plain); add form = floor(Q/t) * m per prime (for lola_add_plain). */
int lola_plain_mul_form(lola_ctx *ctx, const uint32_t *pt_dev, uint32_t *out_dev, lola_stream stream);
int lola_plain_add_form(lola_ctx *ctx, const uint32_t *pt_dev, uint32_t *out_dev, lola_stream stream);

/* Exact integers from residues modulo several plaintext moduli (Chinese
 * remainder theorem; Sec. 4.4 combines the CIFAR network's three plaintext
 * moduli this way).  residues_dev: k device arrays of n int64 values, array i
 * taken mod moduli[i] (e.g. decoded slots of the same network run under each
 * t_i).  moduli: k (1..16) pairwise coprime host values in [2, 2^26).
 * out_dev: n * words int64 (device): value j is the integer X with
 * X = r_i mod t_i for every i and -M/2 <= X < M/2, M = prod t_i, as
 * little-endian two's complement in `words` (1..8) 64-bit words.  Needs
 * M < 2^(64 words), else LOLA_E_INVAL.  No context: the call only enqueues a
 * kernel on `stream` of the current device. */
int lola_crt_combine(const int64_t *const *residues_dev, const uint32_t *moduli, uint32_t k, uint32_t n,
                     int64_t *out_dev, uint32_t words, lola_stream stream);

/* ------------------------------------------------------ encrypt / decrypt */
/* Encryption E of Sec. 3.1: c = (pk0 u + e1 + floor(Q/t) m, pk1 u + e2), u
 * ternary, e1, e2 errors drawn with the seed and the object id `nonce`.
 * pt_dev: N words in [0, t) (lola_encode output); ct_dev: [2][L][N] written.
 * Errors: LOLA_E_INVAL (null pointer). */
int lola_encrypt(lola_ctx *ctx, const uint32_t *pk_dev, const uint32_t *pt_dev, uint64_t seed,
                 uint32_t nonce, uint32_t *ct_dev, lola_stream stream);
/* Decryption D of Sec. 3.1: m_k = round(t x_k / Q) mod t, x = c0 + c1 s
 * (+ c2 s^2) mod Q, computed exactly (mixed-radix, no floating point).
 * size = 2 or 3; pt_dev: N words written.  Errors: LOLA_E_INVAL (null
 * pointer, size not 2 or 3). */
int lola_decrypt(lola_ctx *ctx, const uint32_t *sk_dev, const uint32_t *ct_dev, uint32_t size,
                 uint32_t *pt_dev, lola_stream stream);
/* The same over n messages stored back to back (pt_dev n * N words, ct_dev
 * n ciphertexts of 2 * L * N words; for decryption, of size * L * N words):
 * message i of lola_encrypt_batch is encrypted with object id nonce0 + i and
 * equals lola_encrypt with that nonce word for word (LOLA_E_INVAL when
 * nonce0 + n exceeds 2^32).  Scratch is taken 16 messages at a time. */
int lola_encrypt_batch(lola_ctx *ctx, const uint32_t *pk_dev, const uint32_t *pt_dev, uint32_t n, uint64_t seed,
                       uint32_t nonce0, uint32_t *ct_dev, lola_stream stream);
int lola_decrypt_batch(lola_ctx *ctx, const uint32_t *sk_dev, const uint32_t *ct_dev, uint32_t n, uint32_t size,
                       uint32_t *pt_dev, lola_stream stream);

/* ------------------------------------------------------------- operations */
/* Homomorphic sum of Sec. 3.1: out = a + b, `size` components (2 or 3);
 * may run in place.  Errors: LOLA_E_INVAL. */
int lola_add(lola_ctx *ctx, const uint32_t *a_dev, const uint32_t *b_dev, uint32_t size,
             uint32_t *out_dev, lola_stream stream);
/* Plaintext sum (Sec. 3.1; biases of Sec. 4.3): out = (c0 + floor(Q/t) m,
 * c1), pt_add_dev from lola_plain_add_form; may run in place. */
int lola_add_plain(lola_ctx *ctx, const uint32_t *ct_dev, const uint32_t *pt_add_dev,
                   uint32_t *out_dev, lola_stream stream);
/* Plaintext product, slot by slot (Sec. 3.1 batching; the point-wise
 * products of Sec. 4.2.2): out = (c0 [m]_t, c1 [m]_t), pt_mul_dev from
 * lola_plain_mul_form; may run in place. */
int lola_mul_plain(lola_ctx *ctx, const uint32_t *ct_dev, const uint32_t *pt_mul_dev,
                   uint32_t *out_dev, lola_stream stream);
/* out = [w]_t * ct (message times scalar, Sec. 4.2.2). */
int lola_mul_scalar(lola_ctx *ctx, const uint32_t *ct_dev, int64_t w, uint32_t *out_dev,
                    lola_stream stream);
/* Homomorphic product of Sec. 3.1 (the square activation of Sec. 4.3):
 * size-3 result d_j = round(t (a (x) b)_j / Q) mod Q for the tensor of the
 * centred lifts, computed exactly.  out3_dev [3][L][N] may not alias an
 * input (LOLA_E_INVAL). */
int lola_mul(lola_ctx *ctx, const uint32_t *a_dev, const uint32_t *b_dev, uint32_t *out3_dev,
             lola_stream stream);
/* Relinearisation, the step that brings a product of Sec. 3.1 back to two
 * components: (d0, d1) + KeySwitch_{s^2 -> s}(d2), rlk_dev from
 * lola_keygen_switch with galois 0.  LOLA_E_NOKEY without a key. */
int lola_relin(lola_ctx *ctx, const uint32_t *rlk_dev, const uint32_t *in3_dev, uint32_t *out_dev,
               lola_stream stream);
/* Rotation of the slot matrix (Sec. 3.1: row swap, column rotation; the
 * rotate-and-sum reductions of Sec. 4.1 and 4.2.2): (sigma_g(c0), 0) +
 * KeySwitch_{sigma_g(s) -> s}(sigma_g(c1)), galois from lola_galois_element,
 * gk_dev from lola_keygen_switch with that element.  Errors: LOLA_E_NOKEY,
 * LOLA_E_INVAL (Galois element 0, even or >= 2N). */
int lola_rotate(lola_ctx *ctx, const uint32_t *gk_dev, uint32_t galois, const uint32_t *ct_dev,
                uint32_t *out_dev, lola_stream stream);
/* n rotations of one ciphertext in_dev [2][L][N], by galois[k] (host, odd,
 * 3 <= g < 2N) under keys[k] (host array of device keys) into out_dev[k]
 * (host array of device [2][L][N], none equal to in_dev), sharing one
 * decomposition (hoisting): the key switch's digits are taken from c1 before
 * the automorphism, sigma_g(|c1|_{q_i}) as integer polynomials, so their
 * transforms to every modulus are computed once for all n.  Each output
 * decrypts to the same slots as lola_rotate's; the words differ from it
 * (Sec. 3.1 rotations; the digits are this library's key-switching reading).
 * Scratch: (2L + (L + K) dnum) N words for the source ((L^2 + 3L) N with one
 * special prime) plus (4L + 2K) N per rotation, in chunks of 128. */
int lola_rotate_hoisted(lola_ctx *ctx, const uint32_t *in_dev, uint32_t n, const uint32_t *galois,
                        const uint32_t *const *keys, uint32_t *const *out_dev, lola_stream stream);

/* Key-switch autotuner.  At N = 16384 the three batched key-switch stages
 * (0 digits, 1 inner product, 2 mod-down) are each compiled in several
 * variants: the radix split of their transforms (stages per register pass,
 * written as digits, e.g. 4433) and the LDS placement (padded or plain).
 * Every variant computes the same words.  lola_ks_variants lists a stage's
 * variants (*count = how many, at most cap written; other N: one default);
 * get / set choose the context's variant per stage (LOLA_E_INVAL for an
 * index past the list).  lola_ks_autotune, stage by stage with the others at
 * their best so far, runs a batch of n_jobs (1..128) rotations on synthetic
 * residues with every variant, checks each one's output words against the
 * default's (LOLA_E_DEVICE on a difference), times the whole key switch
 * reps times, and keeps the fastest per stage in the context (chosen[3]),
 * where a variant displaces the one before it only when at least 1% faster.
 * out receives one entry per variant timed, stages in order (ms = average
 * time of the batch); it allocates and synchronises. */
typedef struct {
    uint32_t stage, index, split, padded;
    float ms;
} lola_ks_variant;
int lola_ks_variants(const lola_ctx *ctx, uint32_t stage, lola_ks_variant *out, uint32_t cap, uint32_t *count);
int lola_ks_get_variant(const lola_ctx *ctx, uint32_t stage, uint32_t *index);
int lola_ks_set_variant(lola_ctx *ctx, uint32_t stage, uint32_t index);
int lola_ks_autotune(lola_ctx *ctx, uint32_t n_jobs, uint32_t reps, lola_ks_variant *out, uint32_t cap,
                     uint32_t *chosen, lola_stream stream);

/* lola_rotate for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same rotation, the same words, computed with the batched key-switch
 * kernels on one job whose scratch, (4L + 2K) N words (K special primes),
 * lies in a fixed device array of the library of (4 x 12 + 2 x 2) x 16384
 * words (3.25 MiB; set up per device when a context is created and held
 * until the process ends) and
 * whose descriptor is passed by value; nothing is allocated and no
 * descriptor is uploaded.  Every call on one GPU shares that array, so calls
 * that overlap on one GPU (two streams, two threads) race: the caller
 * orders them.  Nothing in the array needs clearing between calls.  Errors:
 * LOLA_E_NOKEY (no key), LOLA_E_INVAL (null pointer, Galois element 0, even
 * or >= 2N, out == ct), LOLA_E_SHAPE (scratch above the fixed size, which no
 * accepted parameter set reaches), LOLA_E_DEVICE. */
int lola_rotate_noalloc(lola_ctx *ctx, const uint32_t *gk_dev, uint32_t galois, const uint32_t *ct_dev,
                        uint32_t *out_dev, lola_stream stream);

/* Batched key switching: n independent rotations / relinearisations in one
 * set of launches (uneven per-ciphertext work is just more descriptors). */
typedef struct {
    const uint32_t *in_dev;  /* rotation: ciphertext [2][L][N]; relin: [3][L][N] */
    const uint32_t *key_dev; /* switching key */
    uint32_t *out_dev;       /* [2][L][N] */
    uint32_t galois;         /* Galois element; 0 = relinearisation */
    uint32_t pad;
} lola_ks_desc;
int lola_keyswitch_batch(lola_ctx *ctx, const lola_ks_desc *descs_host, uint32_t n,
                         lola_stream stream);

/* Batched forms (host arrays of n device pointers; one launch set):
 * out[k] = ct[k] * pt_mul[k] (mul form), and exact products out3[k] =
 * a[k] x b[k] (outputs may not alias inputs). */
int lola_mul_plain_batch(lola_ctx *ctx, uint32_t n, const uint32_t *const *ct, const uint32_t *const *pt_mul,
                         uint32_t *const *out, lola_stream stream);
int lola_mul_batch(lola_ctx *ctx, uint32_t n, const uint32_t *const *a, const uint32_t *const *b,
                   uint32_t *const *out3, lola_stream stream);

/* Chains of rotations with uneven lengths in one persistent launch: chain k
 * applies its n_steps rotations in order, x <- rotate(x, galois[r]) with
 * keys[r], starting from in_dev and leaving the result in out_dev (tmp_dev is
 * a ping-pong buffer; all three distinct, [2][L][N] each).  n_wg workgroups
 * (0 = 256) each take the next chain from a work counter, longest chains
 * first, and run its rotations as complete key switches; they exit when the
 * counter passes n.  galois and keys are host arrays of n_steps entries. */
typedef struct {
    const uint32_t *in_dev;
    uint32_t *out_dev;
    uint32_t *tmp_dev;
    uint32_t n_steps;
    const uint32_t *galois;          /* host [n_steps] */
    const uint32_t *const *keys;     /* host [n_steps] device pointers */
} lola_chain;
int lola_rotate_chains(lola_ctx *ctx, const lola_chain *chains, uint32_t n, uint32_t n_wg, lola_stream stream);

/* ------------------------------------------------------ canonical forms */
/* Device form <-> coefficient form for n_polys polynomials [n][L][N]. */
int lola_to_coeff(lola_ctx *ctx, const uint32_t *in_dev, uint32_t n_polys, uint32_t *out_dev,
                  lola_stream stream);
int lola_from_coeff(lola_ctx *ctx, const uint32_t *in_dev, uint32_t n_polys, uint32_t *out_dev,
                    lola_stream stream);
/* Keys in coefficient form: secret [L+K][N] (residues of the ternary s),
 * public [2][L][N], switching [dn][2][L+K][N]. */
int lola_export_sk(lola_ctx *ctx, const uint32_t *sk_dev, uint32_t *out_dev, lola_stream stream);
int lola_export_pk(lola_ctx *ctx, const uint32_t *pk_dev, uint32_t *out_dev, lola_stream stream);
int lola_export_ksk(lola_ctx *ctx, const uint32_t *ksk_dev, uint32_t *out_dev, lola_stream stream);

/* Diagnostic: forward or inverse NTT of n limbs, limb k modulo prime index
 * prime_idx_host[k] (0..L-1 ciphertext primes, L..L+K-1 the special primes,
 * L+K..L+K+n_aux-1 the auxiliary primes, L+K+n_aux = t), natural
 * coefficient order <-> bit-reversed evaluation order:
 * out[k] = a(psi^(2 brv(k) + 1)) with psi the smallest primitive 2N-th root.
 * When prime_idx_host[k] = k mod L for every k (the limbs of consecutive
 * polynomials) the launch carries no per-limb descriptors; any other list
 * is uploaded as descriptors first.  The results are the same. */
int lola_ntt_limbs(lola_ctx *ctx, const uint32_t *in_dev, uint32_t *out_dev, uint32_t n_limbs,
                   const uint32_t *prime_idx_host, int inverse, lola_stream stream);

/* Batched NTT variants and their autotuner.  The batched limb transforms
 * (lola_ntt_limbs, lola_to_coeff / lola_from_coeff, encoding, key generation
 * and the executor's transforms) run one compiled variant per context:
 *   split          how the log2(N) butterfly stages group into register
 *                  passes, as decimal digits, first pass first (4442 at
 *                  N = 16384: passes of 4, 4, 4 and 2 stages; one LDS
 *                  exchange between passes);
 *   limbs_per_wg   transforms each workgroup runs in turn (1, 2 or 4).
 * Every variant gives the same words.  Variant 0 is the default.
 * lola_ntt_variants lists them (count = how many; at most cap written; ms
 * = 0).  lola_ntt_set_variant / _get_variant select by index.
 * lola_ntt_autotune times every variant on the context's device: n_limbs
 * limbs of pseudo-random residues (limb k modulo prime k mod L), one forward
 * and one inverse batch per repetition, reps repetitions, timed with HIP
 * events on `stream`; each variant's output is first compared with the
 * default's (LOLA_E_DEVICE if any word differs).  It keeps the fastest
 * (forward + inverse) as the context's variant, writes the index to *chosen
 * and up to cap entries {split, limbs_per_wg, ms per repetition} to out.  It
 * allocates 4 n_limbs N words of device scratch for the duration and
 * synchronises `stream`. */
typedef struct {
    uint32_t split;
    uint32_t limbs_per_wg;
    float ms;
} lola_ntt_variant;
int lola_ntt_variants(const lola_ctx *ctx, lola_ntt_variant *out, uint32_t cap, uint32_t *count);
int lola_ntt_get_variant(const lola_ctx *ctx, uint32_t *index);
int lola_ntt_set_variant(lola_ctx *ctx, uint32_t index);
int lola_ntt_autotune(lola_ctx *ctx, uint32_t n_limbs, uint32_t reps, lola_ntt_variant *out, uint32_t cap,
                      uint32_t *chosen, lola_stream stream);

/* ------------------------------------------------------- layer compiler */
/* Lowers a layer list onto the operations above with the paper's vector
 * representations and matrix-vector recipes (Sec. 4.2: dense, sparse,
 * stacked, interleaved and convolution representations; dense-row-major,
 * stacked-row-major, interleaved-row-major and convolution-row-major
 * products; Sec. 4.3 / Table 1 and App. C / Table 3 for the MNIST pipeline).
 * Supported layer patterns (anything else returns LOLA_E_UNSUPPORTED):
 *   CONV2D, SQUARE, DENSE, SQUARE, DENSE   convolution representation input
 *       (k*k messages), maps combined by rotations, stacked-row-major dense
 *       producing an interleaved vector, interleaved-row-major output layer
 *       (one message per output, value at slot 0);
 *   CONV2D_DENSE_INPUT, SQUARE, DENSE, SQUARE, DENSE   (LoLa-Dense, App. C)
 *       the input is one dense message (padded pixel (i, j) at slot
 *       i*in_w + j); the k*k convolution messages are made from it by
 *       rotations and one 0/1 mask of the window corners; stride 2 only;
 *       maps are combined into the four parity classes of the corner lattice
 *       (and bands below), then stacked as above;
 *   CONV2D, SQUARE, CONV2D, SQUARE, DENSE   (the collapsed CIFAR network of
 *       Sec. 4.4 / App. D) convolution representation of every channel
 *       (channels*k*k messages), maps placed in blocks of n1*n1 slots (as
 *       many per slot row as fit, both rows per message, more messages if
 *       needed) and squared; the second convolution as dense vector - row
 *       major: per output the products with its weights, a sum over the
 *       whole message (rotations 1 .. N/4 and the row swap), then the one-hot
 *       product that keeps slot j; the outputs summed into one message,
 *       squared, and one message per logit (value at slot 0);
 *   CONV2D, SQUARE, CONV2D, then any other chain of DENSE and SQUARE
 *       layers: the same two-convolution front end up to the second
 *       convolution's dense output (value j at slot j), then the chain as
 *       in a dense chain (below);
 *   CONV2D, SQUARE, DENSE   (the small variant of Sec. 4.3) the same front
 *       end, then one stacked-row-major round as the output layer (out_dim <=
 *       N / period): one message, output o at slot period*o;
 *   CONV2D (or CONV2D_DENSE_INPUT), SQUARE, DENSE, then any other chain of
 *       DENSE and SQUARE layers: the same front end and stacked-row-major
 *       rounds up to the interleaved hidden vector, then every further dense
 *       layer with the recipe its input's representation calls for, as in a
 *       dense chain (below): dense vector - row major on the interleaved or
 *       dense vector (a sparse result), sparse vector - column major on a
 *       sparse one (a dense result);
 *   DENSE [, SQUARE]   with in_dim <= N/4: stacked input (period = next power
 *       of two >= in_dim), one row per block, output j at slot period*j;
 *   DENSE, SQUARE, DENSE   with in_dim <= N/2, two recipes (see
 *       lola_compile_ex): stacked-row-major with one query per message (the
 *       client sends N/period copies; rounds, interleaved hidden vector,
 *       interleaved-row-major output, value at slot 0), or dense-row-major with
 *       N/period queries per message (query q in the block at period*q),
 *       hidden units masked and combined into an interleaved vector, then
 *       one message per output with query q's value at slot period*q.
 * Weights and biases are integers, used modulo t. */
enum { LOLA_LAYER_CONV2D = 1, LOLA_LAYER_DENSE = 2, LOLA_LAYER_SQUARE = 3, LOLA_LAYER_CONV2D_DENSE_INPUT = 4 };
typedef struct {
    int32_t kind;
    int32_t in_h, in_w;        /* CONV2D*: input size as the client pads it (square) */
    int32_t k, stride, maps;   /* CONV2D: window, stride, output maps */
    int32_t in_dim, out_dim;   /* DENSE; CONV2D: in_dim = input channels (0 = 1) */
    const int64_t *weight;     /* host; CONV2D [maps][channels][k][k], DENSE [out_dim][in_dim] */
    const int64_t *bias;       /* host; [maps] or [out_dim]; NULL = none */
} lola_layer;

typedef struct lola_plan lola_plan;
typedef struct {
    uint32_t n_inputs, n_outputs, n_ops, n_consts, n_galois, n_waves, queries;
    uint32_t n_rotations, n_mul_plain, n_mul_scalar, n_square, n_add_plain, n_add;
    uint32_t n_phys_regs;      /* device ciphertext buffers per request */
    uint32_t recipe;           /* LOLA_RECIPE_* used for the network's dense layers */
    float predicted_us;        /* cost model: one request (all its queries) inside a large batch, MI355X */
    float predicted_latency_us; /* cost model: one request alone (waves in turn), MI355X */
    uint32_t sums;             /* LOLA_SUMS_SEQUENTIAL or LOLA_SUMS_HOISTED (lola_compile_options) */
} lola_plan_info;

/* Representation choice.  Where more than one recipe applies (candidates
 * below), the compiler builds each candidate, prices it with a per-operation
 * cost model (key switches, products and element-wise passes timed on MI355X
 * at N = 16384, L = 7, scaled by N and L) and keeps the cheapest for the
 * objective: THROUGHPUT = least time per query with full messages
 * (predicted_us / queries), LATENCY = least time for one request alone
 * (predicted_latency_us: waves in turn, each launch priced by its rounds of
 * workgroups over the CUs).  recipe forces one (an inapplicable one gives
 * LOLA_E_UNSUPPORTED).  lola_compile = AUTO, THROUGHPUT. */
enum { LOLA_OBJECTIVE_THROUGHPUT = 0, LOLA_OBJECTIVE_LATENCY = 1 };
/* Candidates:
 *  - Any other chain of DENSE and SQUARE layers (DENSE first, sizes <= N),
 *    one query per message (Sec. 4.2.2): each dense layer takes the recipe
 *    its input's representation calls for -- dense vector - row major on a
 *    dense input (per row a product and a whole-message rotate-and-sum, so
 *    every slot holds the output: one message per row, sparse), sparse
 *    vector - column major on a sparse input (W v = sum_i v_i c^i: one
 *    product per input with column i at slots 0..r-1, summed; dense output,
 *    no rotation); a square squares every message.  DENSE_CHAIN: the client
 *    sends one dense message (value i at slot i); SPARSE_COLUMN_MAJOR: the
 *    client sends in_dim messages, message i holding value i in every slot
 *    (input map).  Outputs: one message (value j at slot j) after a column
 *    major layer, one message per value (at slot 0, and every other slot)
 *    after a row major one.  Both can be forced on any such chain.
 *  - DENSE, SQUARE, DENSE with in_dim <= N/2 (Sec. 4.2.2): DENSE_ROW_MAJOR
 *    (dense vector - row major, N/period queries per message) or
 *    STACKED_ROW_MAJOR (stacked vector - row major, one query per message).
 *  - CONV2D or CONV2D_DENSE_INPUT, SQUARE, DENSE and at least one more
 *    layer, e.g. SQUARE, DENSE (Sec. 4.3, App. C): FULL_REDUCTION, the layout the paper describes (every stacked
 *    round summed over its whole block, masked and combined; one output
 *    message per class: 154 rotations for the MNIST network), or
 *    SHARED_REDUCTION (each round summed only within groups of
 *    next_pow2(rounds) slots, masked to the group starts, combined, then one
 *    rotate-and-sum over the rest of the block for all rounds together; the
 *    last layer on shifted copies of its input into one packed message, class
 *    o at slot next_pow2(rounds)*o: 58 rotations for the MNIST network).  Both
 *    give the same values at the valid slots of every layer.  With a longer
 *    chain after the first dense layer, the recipe chooses that layer's
 *    reduction; the rest of the chain is compiled as a dense chain.
 *  - Everything else: FIXED. */
enum { LOLA_RECIPE_AUTO = 0, LOLA_RECIPE_DENSE_ROW_MAJOR = 1, LOLA_RECIPE_STACKED_ROW_MAJOR = 2,
       LOLA_RECIPE_FIXED = 3 /* reported for patterns with a single recipe */,
       LOLA_RECIPE_FULL_REDUCTION = 4, LOLA_RECIPE_SHARED_REDUCTION = 5,
       LOLA_RECIPE_DENSE_CHAIN = 6, LOLA_RECIPE_SPARSE_COLUMN_MAJOR = 7 };
/* Form of the rotate-and-sum reductions and shifted combinations
 * (Sec. 4.2.2).  SEQUENTIAL: x += rot(x, s) step by step, and binary trees of
 * rotate-and-adds: the fewest rotations, one level each.  HOISTED (a layout
 * for single requests, where the GPU is mostly idle and the depth sets the
 * latency): consecutive steps other than the row swap in groups of up to
 * three, each group the 2^k - 1 rotations of the current message by the
 * group's subset sums, hoisted (one decomposition for all), added to it in
 * one linear combination; combinations of shifted messages in one level (every
 * member rotated by its own offset, then one linear combination).  The same
 * slots, more rotations (and keys), fewer levels.  AUTO: SEQUENTIAL for the
 * throughput objective; for the latency objective both are built and priced
 * with every candidate recipe. */
enum { LOLA_SUMS_AUTO = 0, LOLA_SUMS_SEQUENTIAL = 1, LOLA_SUMS_HOISTED = 2 };
typedef struct {
    int32_t objective;
    int32_t recipe;
    int32_t sums;              /* LOLA_SUMS_* */
} lola_compile_options;

int lola_compile(const lola_params *params, const lola_layer *layers, uint32_t n_layers, lola_plan **out);
int lola_compile_ex(const lola_params *params, const lola_layer *layers, uint32_t n_layers,
                    const lola_compile_options *options, lola_plan **out);
void lola_plan_destroy(lola_plan *plan);
int lola_plan_get_info(const lola_plan *plan, lola_plan_info *info);
/* Galois elements of the rotation keys the plan needs, in the order
 * lola_request.gk_dev must follow. */
int lola_plan_galois(const lola_plan *plan, uint32_t *galois_host);
/* map[m*N + s] = index of the input value the client places at slot s of
 * input message m (queries concatenated), or -1 for a zero slot. */
int lola_plan_input_map(const lola_plan *plan, int32_t *map_host);
/* map[o*N + s] = index of the result value at slot s of output message o
 * (query-major: q*out_dim + j), or -1. */
int lola_plan_output_map(const lola_plan *plan, int32_t *map_host);
/* The op list as text, one op per line (for inspection and tests):
 *   lincomb DST SRC:W ... [+add CONST]   sum of scalar multiples (+ add-form constant)
 *   mulplain DST SRC CONST [+add CONST]  product with a plaintext (+ add-form constant)
 *   addplain DST SRC CONST
 *   rotadd DST SRC STEP ADDEND           ADDEND + rotate(SRC, STEP) (STEP "swap" = row swap)
 *   rot DST SRC STEP
 *   square DST SRC
 * followed by "outputs R ...".  Registers 0..n_inputs-1 are the inputs.
 * Returns the needed size (with the terminating zero) if cap is too small. */
int lola_plan_dump(const lola_plan *plan, char *buf, size_t cap);
/* The N slot values of plaintext constant `id` (as in the dump). */
int lola_plan_const(const lola_plan *plan, uint32_t id, int64_t *slots_host);
/* Encodes the plan's constants on the context's device (plaintext mul /
 * add forms).  Needed once before evaluation. */
int lola_plan_load(lola_ctx *ctx, lola_plan *plan, lola_stream stream);

typedef struct {
    const uint32_t *rlk_dev;          /* relinearisation key */
    const uint32_t *const *gk_dev;    /* host array [n_galois] of switching keys */
    const uint32_t *const *in_dev;    /* host array [n_inputs] of ciphertexts */
    uint32_t *const *out_dev;         /* host array [n_outputs] of ciphertexts */
} lola_request;
/* Evaluates the plan for n_req independent requests (each with its own keys
 * and inputs).  Ops are grouped into waves of independent operations; every
 * op kind of a wave runs as one batched launch over all requests.  Output
 * buffers must not alias inputs.  The plan owns its device workspace
 * (ciphertext registers and scratch), sized for the largest n_req seen.
 * Batches of 16 or more requests run as two lanes: the first half on
 * `stream`, the second on a stream the plan owns (non-blocking, default
 * priority) that waits for `stream`'s earlier work and is waited for by it,
 * so the call stays ordered on `stream` like a single-stream one.  Each lane
 * has its own workspace.  With kernel timing on (lola_timing_enable), or
 * after lola_plan_set_lanes(plan, 1), a batch runs as one lane. */
int lola_evaluate(lola_ctx *ctx, lola_plan *plan, const lola_request *reqs, uint32_t n_req,
                  lola_stream stream);
/* Upper bound on the lanes of lola_evaluate: 1 or 2 (the default). */
int lola_plan_set_lanes(lola_plan *plan, uint32_t max_lanes);
/* Same, replayed through a HIP graph captured on the first call for this
 * exact set of buffers (re-captured when any pointer, n_req or the number of
 * lanes changes).  A batch of 16 or more requests is captured as two lanes,
 * forked onto the plan's second stream and joined back inside the graph. */
int lola_evaluate_graph(lola_ctx *ctx, lola_plan *plan, const lola_request *reqs, uint32_t n_req,
                        lola_stream stream);

/* ---------------------------------------------------------------- serving */
/* A request loop with continuous batching (a server holding encrypted
 * queries, keys and intermediate ciphertexts on the device).  Models are
 * loaded plans, one per ring size; each runs on its own stream with a pool of
 * request slots.  Admission is by HBM footprint: a model gets as many slots
 * (register file + temporaries of one request) as fit in the remaining
 * budget, up to max_inflight; a queued request enters when a slot is free.
 * Every lola_server_step admits queued requests and issues, per model, the
 * next wave of all its in-flight requests as one batched launch set, so
 * requests that arrive while others are on the GPU join them at once.  A
 * model granted 16 or more slots (and a second scratch area within the
 * budget) runs a round of 16 or more requests as two lanes: half of them on
 * a second stream, forked and joined within the round.  The
 * caller keeps a request's buffers alive until its tag is returned by
 * lola_server_poll.  Results equal those of lola_evaluate on the request
 * alone, word for word. */
typedef struct lola_server lola_server;
int lola_server_create(size_t hbm_budget_bytes, lola_server **out);
void lola_server_destroy(lola_server *srv);
int lola_server_add_model(lola_server *srv, lola_ctx *ctx, lola_plan *plan, uint32_t max_inflight,
                          uint32_t *model_id);
/* Slots granted, HBM bytes per slot, the model's scratch bytes (both lanes'), jobs launched. */
int lola_server_model_info(const lola_server *srv, uint32_t model_id, uint32_t *slots, uint64_t *footprint_bytes,
                           uint64_t *scratch_bytes, uint64_t *launched_jobs);
int lola_server_submit(lola_server *srv, uint32_t model_id, const lola_request *req, uint64_t tag);
/* A solo plan for a model: the same network compiled for one request alone
 * (lola_compile_ex with the latency objective; more rotations in fewer
 * levels), loaded on the model's context, with the same input and output
 * maps as the model's plan.  It gets one slot of its own (charged to the
 * budget).  A request submitted with keys for it (lola_server_submit_ex) that
 * finds the model idle -- nothing else in flight or queued -- runs under the
 * solo plan; requests arriving meanwhile run under the model's plan, their
 * waves in the same rounds.  Set before any request is submitted
 * (LOLA_E_INVAL otherwise; LOLA_E_SHAPE for other maps, LOLA_E_NOMEM past the
 * budget).  A result's words are those of lola_evaluate on the request alone
 * under the plan that served it (lola_server_poll_ex says which); both
 * decrypt to the same values. */
int lola_server_set_solo_plan(lola_server *srv, uint32_t model_id, lola_plan *solo);
/* lola_server_submit with the Galois keys of the solo plan (in the order of
 * its lola_plan_galois; NULL: the request always runs under the model's
 * plan).  The request's other buffers serve both plans. */
int lola_server_submit_ex(lola_server *srv, uint32_t model_id, const lola_request *req,
                          const uint32_t *const *solo_gk_dev, uint64_t tag);
/* One scheduling round (non-blocking except to keep two rounds in flight per
 * model); *pending = queued + in-flight requests. */
int lola_server_step(lola_server *srv, uint32_t *pending);
/* Tags of requests completed since the last poll (at most cap). */
int lola_server_poll(lola_server *srv, uint64_t *tags, uint32_t cap, uint32_t *n);
/* As lola_server_poll, with the plan that served each request in forms[i]
 * (forms may be NULL). */
enum { LOLA_SERVED_PLAN = 0, LOLA_SERVED_SOLO = 1 };
int lola_server_poll_ex(lola_server *srv, uint64_t *tags, uint32_t *forms, uint32_t cap, uint32_t *n);

/* Kernel timing (for measurement).  While enabled, the library records a HIP
 * event pair on the launch stream around every launch of its hot-path
 * kernels: the batched NTT, each key-switch stage, the three product stages,
 * the linear-combination and plaintext kernels and the persistent chain
 * kernel.  Events between launches serialise them, so timed passes measure
 * launches alone (plans then run one lane).  Both readers below synchronise
 * on the recorded events, then clear every total. */
int lola_timing_enable(lola_ctx *ctx, int on);
/* The key-switch inner-product stage (ks_inner, or the latency forms'
 * term/fold kernels): summed ms, launches, and key switches issued. */
int lola_kernel_timing(lola_ctx *ctx, double *total_ms, uint64_t *launches, uint64_t *jobs);
/* Per kernel: summed event time, launches, work units, and the algorithmic
 * HBM bytes and VALU lane-ops the library charges for them.  Bytes count
 * each distinct buffer a launch reads once (jobs of a batch share keys,
 * sources and constants); lane-ops count every job's work.  Units and the
 * charges (N ring degree, L ciphertext primes, K special primes, dn digits,
 * M = L + K, T = 9 (N/2) log2 N lane-ops of one limb transform, KB = 8N dn M
 * bytes of one switching key, X = dn M - L transformed (target, digit)
 * pairs, G of them with a two-prime digit, 14 lane-ops per Garner step; with
 * K = 1: dn = L, X = L^2, G = 0):
 *   ntt_jobs_kernel          limb             8N B,  T
 *   ks_digits_kernel         (job, prime)     12N B, T
 *   ks_inner_kernel          job              KB per distinct key + 8N (2L+K) B,
 *                                             (X + 2K) T + 14 dn M N + 14 G N
 *   ks_moddown_kernel        (job, prime, component)  (12 + 4K) N B, T + 10N (+ 14N if K = 2)
 *   ks_modup_kernel          source           8N X + 4N G B, X T + 14 G N
 *   ks_digits_kernel/hoist, ks_moddown_kernel/hoist: the same kernels run
 *                            for hoisted rotations, charged as above
 *   ks_hoisted_inner_kernel  rotation         KB per distinct key + 4N dn M per distinct
 *                            source + 8N (L+K) B, 2K T + 14 dn M N
 *   tensor_*_kernel, lin_kernel, plain_kernel, latency-form and chain
 *   kernels: as documented at their launch sites.
 * Writes at most cap entries (kernels with no launch are skipped) and sets
 * *n_out to the number of kernels with launches; returns LOLA_E_INVAL when
 * that exceeds cap.  `name` points to a static string. */
typedef struct {
    const char *name;
    double total_ms;
    uint64_t launches;
    uint64_t units;
    double alg_bytes;
    double alg_ops;
} lola_kernel_stat;
int lola_kernel_stats(lola_ctx *ctx, lola_kernel_stat *out, uint32_t cap, uint32_t *n_out);

/* VALU issue-rate probe, for stating the integer peak the kernels are
 * measured against: op 0 v_mul_lo_u32, 1 v_mul_hi_u32, 2 v_add_u32, each
 * thread running eight independent chains of `iters` x 16 steps of the one
 * instruction, 8 workgroups of 256 threads per compute unit.  out_dev is a
 * device buffer of out_words >= 2048 x (compute units) words that the probe
 * overwrites (values meaningless).  *lane_ops_per_s receives the achieved
 * rate (lane-instructions per second, HIP events on `stream`); synchronises.
 * Errors: LOLA_E_INVAL (bad op, null pointer, iters 0), LOLA_E_SHAPE (buffer
 * too small), LOLA_E_DEVICE. */
int lola_valu_probe(int op, uint32_t iters, uint32_t *out_dev, uint32_t out_words, double *lane_ops_per_s,
                    lola_stream stream);

const char *lola_strerror(int code);
const char *lola_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LOLA_H */
