// Internal definitions of the LoLa BFV library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/lola.h"
#include "modarith.hpp"

namespace lola {

constexpr int MAXL = 12;   // ciphertext primes
constexpr int MAXK = 2;    // special primes of key switching
constexpr int MAXB = 14;   // auxiliary primes of the exact ct x ct product

// Constants of the exact mixed-radix conversions, on the device.
//   Q basis: primes q_0..q_{L-1};  B basis: primes b_0..b_{nB-1}.
struct MrcConst {
    uint32_t L, nB, t, K;
    // Garner: q_k^-1 mod q_i (k < i), Shoup pairs.   [i][k]
    uint32_t invQ[MAXL][MAXL], invQp[MAXL][MAXL];
    // W_k = q_0...q_{k-1} reduced mod b_j, Shoup pairs. [j][k]
    uint32_t wQb[MAXB][MAXL], wQbp[MAXB][MAXL];
    // W_k mod t (decrypt) [k]
    uint32_t wQt[MAXL], wQtp[MAXL];
    // MRC digits of (Q-1)/2
    uint32_t hQ[MAXL];
    // Q mod b_j and Q^-1 mod b_j (Shoup pairs)
    uint32_t Qb[MAXB], Qbp[MAXB], Qinvb[MAXB], Qinvbp[MAXB];
    // t mod q_i, t mod b_j (Shoup pairs)
    uint32_t tq[MAXL], tqp[MAXL], tb[MAXB], tbp[MAXB];
    // Q^-1 mod t (Shoup pair), Delta = floor(Q/t) mod q_i (Shoup pairs)
    uint32_t Qinvt, Qinvtp;
    uint32_t deltaq[MAXL], deltaqp[MAXL];
    // B-side Garner: b_k^-1 mod b_j (k < j)   [j][k]
    uint32_t invB[MAXB][MAXB], invBp[MAXB][MAXB];
    // V_k = b_0...b_{k-1} mod q_i   [i][k]
    uint32_t wBq[MAXL][MAXB], wBqp[MAXL][MAXB];
    uint32_t hB[MAXB];            // MRC digits of (B-1)/2
    uint32_t Bq[MAXL];            // B mod q_i
    // key switching: P = p_0 ... p_{K-1} mod q_i (Shoup), P^-1 mod q_i (Shoup)
    uint32_t Pq[MAXL], Pqp[MAXL], Pinvq[MAXL], Pinvqp[MAXL];
    // two special primes: p_1, p_0^-1 mod p_1 (Shoup), (p_0 - 1)/2, (p_1 - 1)/2,
    // p_0 mod q_i (Shoup)
    uint32_t sp1, sp_inv, sp_invp, sp_half0, sp_half1;
    uint32_t p0q[MAXL], p0qp[MAXL];
    // digits of two ciphertext primes a = 2d, b = 2d + 1: q_b, q_a^-1 mod q_b
    // (Shoup), and q_a mod every key-switching modulus m (Shoup)
    uint32_t gqb[MAXL / 2], ginv[MAXL / 2], ginvp[MAXL / 2];
    uint32_t gq[MAXL / 2][MAXL + MAXK], gqp[MAXL / 2][MAXL + MAXK];
};

// Kernels whose launches the library times when kernel timing is on, each
// with its unit of work (what `units` counts) and the algorithmic HBM bytes and
// VALU lane-ops the launch site charges per unit.
enum KernelId : uint32_t {
    KID_NTT,               // one limb transform
    KID_KS_DIGITS,         // one (key switch, digit)
    KID_KS_INNER,          // one key switch
    KID_KS_MODDOWN,        // one (key switch, prime, component)
    KID_KS_TERM,           // one key switch (latency form)
    KID_KS_FOLD,           // one key switch (latency form)
    KID_KS_TERM_DIRECT,    // one key switch (two-kernel latency form)
    KID_KS_FOLD_MODDOWN,   // one key switch (two-kernel latency form)
    KID_KS_MODUP,          // one hoisting source
    KID_KS_HOISTED_INNER,  // one hoisted rotation
    KID_TENSOR_EXTEND,     // one ciphertext pair
    KID_TENSOR_PRODUCT,    // one ciphertext pair
    KID_TENSOR_ROUND,      // one ciphertext pair
    KID_LIN,               // one linear combination
    KID_PLAIN,             // one plaintext product / add
    KID_CHAIN,             // one rotation of the persistent chain kernel
    KID_KS_HOIST_DIGITS,   // ks_digits_kernel for hoisting sources: one (source, digit)
    KID_KS_HOIST_MODDOWN,  // ks_moddown_kernel for hoisted rotations: one (rotation, prime, component)
    KID_COUNT
};
struct TimedLaunch {
    uint32_t kid;
    uint64_t units;
    double bytes, ops;
    hipEvent_t a, b;
};
struct KernelTotal {
    double ms = 0, bytes = 0, ops = 0;
    uint64_t launches = 0, units = 0;
};

}  // namespace lola

// Prime index layout inside a context: [0, L) ciphertext primes, [L, L+K)
// the special primes of key switching, [L+K, L+K+nB) auxiliary primes,
// L+K+nB = plaintext modulus t.
struct lola_ctx {
    int device = 0;
    uint32_t N = 0, logN = 0;
    uint32_t L = 0, nB = 0;
    uint32_t K = 1;                      // special primes (digits of K ciphertext primes)
    uint32_t t = 0;
    std::vector<uint32_t> primes;        // all moduli, layout above
    std::vector<lola::ModConst> mc_host;
    lola::MrcConst mrc_host{};
    // device tables
    lola::ModConst *d_mc = nullptr;
    lola::MrcConst *d_mrc = nullptr;
    lola::TwPair *d_tw = nullptr, *d_itw = nullptr;   // [nprimes][N] (twiddle, Shoup companion)
    uint32_t *d_slotpos = nullptr;       // slot s -> spectral index mod t
    // scratch arena
    void *d_scratch = nullptr;
    size_t scratch_bytes = 0;
    // descriptor staging for batched launches: a pinned host ring copied to a
    // device ring; slabs are reused once the event recorded when leaving them
    // has completed.
    static constexpr int RING_SLABS = 16;
    static constexpr size_t RING_SLAB = 1024 * 1024;
    uint8_t *h_ring = nullptr, *d_ring = nullptr;
    size_t ring_off = 0;
    hipEvent_t ring_ev[RING_SLABS] = {};
    bool ring_ev_valid[RING_SLABS] = {};
    // kernel timing: an event pair around every timed kernel launch, resolved
    // into per-kernel totals when read
    bool timing = false;
    std::vector<lola::TimedLaunch> timed;    // launches not yet resolved
    std::vector<hipEvent_t> timing_pool;     // free events
    lola::KernelTotal ktot[lola::KID_COUNT];
    uint64_t timed_jobs = 0;                 // key switches issued while timing
    // batched NTT variant (index into the variant list of this N; 0 = default)
    uint32_t ntt_variant = 0;
    // ChaCha20 key words 2..7 of every random stream (words 0, 1: the call's seed)
    uint32_t key_hi[6] = {0, 0, 0, 0, 0, 0};
    // batched key-switch stage variants (0 digits, 1 inner, 2 mod-down; 0 = default)
    uint32_t ks_var[3] = {0, 0, 0};
    uint32_t idxP() const { return L; }
    uint32_t idxB(uint32_t j) const { return L + K + j; }
    uint32_t idxT() const { return L + K + nB; }
    uint32_t nprimes() const { return L + K + 1 + nB; }
    uint32_t dnum() const { return (L + K - 1) / K; }   // key-switching digits
};

namespace lola {

// error reporting (thread-local message)
int set_error(int code, const std::string &msg);
int check_hip(hipError_t e, const char *what);
#define LOLA_HIP(call)                                         \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return ::lola::check_hip(_e, #call); \
    } while (0)

// scratch arena (device); grows with a device synchronisation
int scratch_get(lola_ctx *ctx, size_t bytes, void **out);
// Takes the device address of the fixed scratch array that
// lola_rotate_noalloc uses, once per device (idempotent).
int noalloc_setup(int device);
// Kernel timing around one launch: ktime_begin records a start event when
// timing is on (*a stays null otherwise); ktime_end records the stop event and
// keeps the launch with its kernel id, units and algorithmic cost.
int ktime_begin(lola_ctx *ctx, hipStream_t s, hipEvent_t *a);
int ktime_end(lola_ctx *ctx, hipStream_t s, hipEvent_t a, uint32_t kid, uint64_t units, double bytes, double ops);
#define LOLA_TIMED(ctx, s, kid, units, bytes, ops, ...)                                      \
    do {                                                                                     \
        hipEvent_t _ta = nullptr;                                                            \
        if ((ctx)->timing) {                                                                 \
            int _tr = ::lola::ktime_begin((ctx), (s), &_ta);                                 \
            if (_tr) return _tr;                                                             \
        }                                                                                    \
        __VA_ARGS__;                                                                         \
        if (_ta) {                                                                           \
            int _tr = ::lola::ktime_end((ctx), (s), _ta, (kid), (units), (bytes), (ops));    \
            if (_tr) return _tr;                                                             \
        }                                                                                    \
    } while (0)

// Algorithmic cost conventions shared by the launch sites (VALU lane-ops):
// a lazy Harvey butterfly is 9 ops (Shoup product 3 multiplies + 1 subtract,
// add, subtract, one conditional correction of 2); a modular product 4; a
// modular add or subtract 2; a key multiply-accumulate 7 (a Montgomery
// product and an add, although the kernels accumulate in 64 bits and reduce
// once).  A limb transform is 9 (N/2) log2 N.
constexpr double COST_BFLY = 9, COST_MUL = 4, COST_ADD = 2, COST_MAC = 7;
// A Garner step (a digit of two primes, or the two special primes, to another
// modulus): two modular products and three adds or reductions.
constexpr double COST_GARNER = 2 * COST_MUL + 3 * COST_ADD;
inline double xform_ops(const lola_ctx *ctx) { return COST_BFLY * (ctx->N / 2) * ctx->logN; }
// descriptor upload area (device), copied asynchronously on the stream
int desc_upload(lola_ctx *ctx, const void *host, size_t bytes, hipStream_t s, void **dev);

// host arithmetic helpers
uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t m);
uint64_t powmod_host(uint64_t a, uint64_t e, uint64_t m);
uint64_t invmod_host(uint64_t a, uint64_t m);
inline uint32_t shoup_companion(uint32_t w, uint32_t q) { return (uint32_t)(((uint64_t)w << 32) / q); }

// automorphism index map in the NTT domain: output index j reads input brv-index
LOLA_HD uint32_t galois_src_index(uint32_t j, uint32_t g, uint32_t logN) {
    uint32_t N = 1u << logN;
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t bj = __brev(j) >> (32 - logN);
#else
    uint32_t bj = 0;
    for (uint32_t b = 0; b < logN; ++b)
        if (j & (1u << b)) bj |= 1u << (logN - 1 - b);
#endif
    uint32_t e = (uint32_t)(((uint64_t)g * (2 * bj + 1)) & (2 * N - 1));
    uint32_t k = (e - 1) >> 1;
#if defined(__HIP_DEVICE_COMPILE__)
    return __brev(k) >> (32 - logN);
#else
    uint32_t r = 0;
    for (uint32_t b = 0; b < logN; ++b)
        if (k & (1u << b)) r |= 1u << (logN - 1 - b);
    return r;
#endif
}

// ---- launch helpers implemented in the .hip files ----
struct NttJob {
    const uint32_t *src;
    uint32_t *dst;
    uint32_t prime;     // prime index in the context
    uint32_t flags;     // NTT_* below
};
enum : uint32_t {
    NTT_INVERSE = 1u,
    NTT_SRC_SIGNED_T = 2u,   // source holds residues mod t; lift centred before reducing
    NTT_SRC_REDUCE = 4u,     // source values may exceed the prime: reduce first
    NTT_TO_MONT = 8u,        // multiply the output by 2^32 (Montgomery form)
    NTT_FROM_MONT = 16u,     // multiply the input by 2^-32 before an inverse transform
    NTT_MUL_DELTA = 32u,     // multiply the forward output by floor(Q/t) mod q (prime < L)
    NTT_SRC_SIGNED32 = 64u,  // source holds small signed int32 values (|v| < q)
};
int launch_ntt_jobs(lola_ctx *ctx, const NttJob *host_jobs, int n, hipStream_t s);
int launch_ntt_jobs_dev(lola_ctx *ctx, const NttJob *d_jobs, int n, hipStream_t s);
// n contiguous limbs, limb k under prime k mod cycle, one flag set: launched
// without descriptors.
int launch_ntt_strided(lola_ctx *ctx, const uint32_t *in, uint32_t *out, uint32_t n, uint32_t cycle,
                       uint32_t flags, hipStream_t s);

// One key switch: out = (add0' + KS(x)_0, add1 + KS(x)_1) (+ addct), where
// add0' is add0 under the automorphism when galois > 1.
struct KsJob {
    const uint32_t *x;      // [L][N] polynomial to switch (NTT form, before sigma_g)
    const uint32_t *key;    // [dn][2][L+K][N] Montgomery NTT form
    const uint32_t *add0;   // [L][N] added to component 0 (sigma_g applied), or null
    const uint32_t *add1;   // [L][N] added to component 1, or null
    const uint32_t *addct;  // [2][L][N] added to both components as is, or null
    uint32_t *out;          // [2][L][N]
    uint32_t *scratch;      // (4L + 2K) N words: D [L][N], Xp [L][N] (term form only), U [2][L][N], UP [2][K][N]
    uint32_t galois;        // 0/1: no automorphism
    uint32_t pad;
    const uint32_t *hoist;  // hoisted rotation: the source's hoist area (ks_hoist_limb), else null
};
// Runs the jobs in chunks (assigns scratch, uploads descriptors).
int keyswitch_host_jobs(lola_ctx *ctx, std::vector<KsJob> &jobs, hipStream_t s);
// Exact products out3[k] = a[k] x b[k] for n pairs.
int mul_batch(lola_ctx *ctx, uint32_t n, const uint32_t *const *a, const uint32_t *const *b,
              uint32_t *const *out3, hipStream_t s);
size_t mul_scratch_words(const lola_ctx *ctx);   // per pair
size_t ks_scratch_words(const lola_ctx *ctx);    // per key switch job, launches of many jobs
size_t ks_launch_words(const lola_ctx *ctx, uint32_t n);     // a launch of n jobs
size_t ks_chunk_words(const lola_ctx *ctx, uint32_t chunk);  // any launch of at most chunk jobs
size_t ks_hoist_words(const lola_ctx *ctx);      // hoist area of one source of hoisted rotations
// Algorithmic lane-ops and HBM bytes of one whole batched key switch (digits,
// inner product, mod-down; ciphertext in and out, one key read).
double ks_whole_ops(const lola_ctx *ctx);
double ks_whole_bytes(const lola_ctx *ctx);

}  // namespace lola
