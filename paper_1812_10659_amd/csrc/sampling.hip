// Randomness (ChaCha20, RFC 8439), key generation, encryption, decryption.
//
// Every random value is a 64-bit word of a ChaCha20 stream: key = (seed lo,
// seed hi, k2, ..., k7) with k2..k7 the context's key words (zero unless set
// with lola_set_key_words), nonce = (domain, object, limb), block counter =
// coefficient / 8, word = coefficient mod 8.  Uniform residues are word mod m,
// ternary values word mod 3 - 1, errors a centred binomial over 2 x 21 bits.
#include <algorithm>
#include <vector>

#include "lola_internal.hpp"
#include "mrc.hpp"

namespace lola {

enum : uint32_t {
    DOM_SK = 1, DOM_PK_A = 2, DOM_PK_E = 3, DOM_KSK_A = 4, DOM_KSK_E = 5,
    DOM_ENC_U = 6, DOM_ENC_E1 = 7, DOM_ENC_E2 = 8
};
enum : uint32_t { SAMPLE_UNIFORM = 0, SAMPLE_TERNARY = 1, SAMPLE_CBD = 2 };

__device__ __forceinline__ uint32_t rotl(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }
#define LOLA_QR(a, b, c, d)                 \
    a += b; d ^= a; d = rotl(d, 16);        \
    c += d; b ^= c; b = rotl(b, 12);        \
    a += b; d ^= a; d = rotl(d, 8);         \
    c += d; b ^= c; b = rotl(b, 7);

struct ChachaKey {
    uint32_t w[8];
};

__device__ void chacha20_block(const ChachaKey &k, uint32_t counter, uint32_t n0, uint32_t n1, uint32_t n2,
                               uint32_t (&out)[16]) {
    const uint32_t s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, k.w[0], k.w[1], k.w[2], k.w[3],
                            k.w[4], k.w[5], k.w[6], k.w[7], counter, n0, n1, n2};
    uint32_t x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = s[i];
#pragma unroll 1
    for (int r = 0; r < 10; ++r) {
        LOLA_QR(x[0], x[4], x[8], x[12]);
        LOLA_QR(x[1], x[5], x[9], x[13]);
        LOLA_QR(x[2], x[6], x[10], x[14]);
        LOLA_QR(x[3], x[7], x[11], x[15]);
        LOLA_QR(x[0], x[5], x[10], x[15]);
        LOLA_QR(x[1], x[6], x[11], x[12]);
        LOLA_QR(x[2], x[7], x[8], x[13]);
        LOLA_QR(x[3], x[4], x[9], x[14]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

struct SampleJob {
    uint32_t *dst;      // N words: uniform residues, or signed int32 values
    uint32_t domain, object, limb, kind;
    uint32_t modulus;   // uniform only
    uint32_t pad;
};

// grid: (N/8 blocks of 8 coefficients / blockDim, jobs)
__global__ void sample_kernel(const SampleJob *__restrict__ jobs, uint32_t N, ChachaKey key) {
    const SampleJob job = jobs[blockIdx.y];
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= N / 8) return;
    uint32_t o[16];
    chacha20_block(key, b, job.domain, job.object, job.limb, o);
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        const uint64_t word = (uint64_t)o[2 * w] | ((uint64_t)o[2 * w + 1] << 32);
        uint32_t v;
        if (job.kind == SAMPLE_UNIFORM) {
            v = (uint32_t)(word % job.modulus);
        } else if (job.kind == SAMPLE_TERNARY) {
            v = (uint32_t)((int32_t)(word % 3) - 1);
        } else {
            v = (uint32_t)(__popcll(word & 0x1FFFFFull) - __popcll((word >> 21) & 0x1FFFFFull));
        }
        job.dst[b * 8 + w] = v;
    }
}

static int launch_samples(lola_ctx *ctx, uint64_t seed, const std::vector<SampleJob> &jobs, hipStream_t s) {
    if (jobs.empty()) return LOLA_OK;
    void *d = nullptr;
    int rc = desc_upload(ctx, jobs.data(), jobs.size() * sizeof(SampleJob), s, &d);
    if (rc) return rc;
    const uint32_t nb = ctx->N / 8;
    ChachaKey key{{(uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0}};
    for (int k = 0; k < 6; ++k) key.w[2 + k] = ctx->key_hi[k];
    hipLaunchKernelGGL(sample_kernel, dim3((nb + 127) / 128, (unsigned)jobs.size()), dim3(128), 0, s,
                       (const SampleJob *)d, ctx->N, key);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

constexpr uint32_t CLIENT_CHUNK = 16;   // messages per scratch fill in encrypt / decrypt

// a*b mod q for residues in normal form (two Montgomery steps).
__device__ __forceinline__ uint32_t mulmod_plain(uint32_t a, uint32_t b, const ModConst &c) {
    return mont_mul(mont_mul(a, b, c.q, c.qneg_inv), c.r2_mod, c.q, c.qneg_inv);
}
__device__ __forceinline__ uint32_t to_mont(uint32_t a, const ModConst &c) {
    return shoup(a, c.r_mod, c.r_shoup, c.q);
}

// pk0 = -(a s + e), pk1 = a, both in Montgomery form.  grid (N/256, L)
__global__ void pk_combine_kernel(const uint32_t *__restrict__ ahat, const uint32_t *__restrict__ ehat,
                                  const uint32_t *__restrict__ sk, uint32_t *__restrict__ pk, uint32_t N,
                                  uint32_t L, const ModConst *__restrict__ mcs) {
    const uint32_t j = blockIdx.y, k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const ModConst c = mcs[j];
    const size_t o = (size_t)j * N + k;
    uint32_t as = mulmod_plain(ahat[o], sk[o], c);
    uint32_t v = sub_mod(0, add_mod(as, ehat[o], c.q), c.q);
    pk[o] = to_mont(v, c);
    pk[(size_t)L * N + o] = to_mont(ahat[o], c);
}

// b_d = -a_d s + e_d + [q_j a prime of digit d] (P mod q_j) s'; stored
// [d][0=b,1=a][j][N], Montgomery.  Digit d holds the K consecutive
// ciphertext primes from d K.  grid (N/256, L+K moduli, dn digits)
__global__ void ksk_combine_kernel(const uint32_t *__restrict__ ahat, const uint32_t *__restrict__ ehat,
                                   const uint32_t *__restrict__ sk, const uint32_t *__restrict__ sprime,
                                   uint32_t *__restrict__ ksk, uint32_t N, uint32_t L, uint32_t K,
                                   const ModConst *__restrict__ mcs, const MrcConst *__restrict__ mrc) {
    const uint32_t j = blockIdx.y, i = blockIdx.z, k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const uint32_t M = L + K;
    const ModConst c = mcs[j];
    const size_t aoff = ((size_t)i * M + j) * N + k;
    const size_t soff = (size_t)j * N + k;
    uint32_t a = ahat[aoff];
    uint32_t v = sub_mod(ehat[aoff], mulmod_plain(a, sk[soff], c), c.q);
    if (j < L && j / K == i) v = add_mod(v, shoup(sprime[soff], mrc->Pq[j], mrc->Pqp[j], c.q), c.q);
    const size_t base = (size_t)i * 2 * M * N;
    ksk[base + (size_t)j * N + k] = to_mont(v, c);
    ksk[base + (size_t)M * N + (size_t)j * N + k] = to_mont(a, c);
}

// s'_j = s_j^2 (relinearisation) or s_j at the Galois source index.
__global__ void sprime_kernel(const uint32_t *__restrict__ sk, uint32_t *__restrict__ sp, uint32_t N,
                              uint32_t logN, uint32_t galois, const ModConst *__restrict__ mcs) {
    const uint32_t j = blockIdx.y, k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const ModConst c = mcs[j];
    const uint32_t *s = sk + (size_t)j * N;
    sp[(size_t)j * N + k] = galois == 0 ? mulmod_plain(s[k], s[k], c) : s[galois_src_index(k, galois, logN)];
}

// c0 = pk0 u + e1 + Delta m, c1 = pk1 u + e2 (NTT domain).  grid (N/256, L)
// grid (N/256, L, messages): message z reads its transformed samples at
// z * msg_words past uh, e1h, e2h and mh, and writes ciphertext z.
__global__ void enc_combine_kernel(const uint32_t *__restrict__ pk, const uint32_t *__restrict__ uh,
                                   const uint32_t *__restrict__ e1h, const uint32_t *__restrict__ e2h,
                                   const uint32_t *__restrict__ mh, size_t msg_words, uint32_t *__restrict__ ct,
                                   uint32_t N, uint32_t L, const ModConst *__restrict__ mcs) {
    const uint32_t j = blockIdx.y, k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const ModConst c = mcs[j];
    const size_t P1 = (size_t)L * N, o = (size_t)j * N + k, om = blockIdx.z * msg_words + o;
    uh += om - o;
    e1h += om - o;
    e2h += om - o;
    mh += om - o;
    ct += blockIdx.z * 2 * P1;
    const uint32_t u = uh[o];
    uint32_t c0 = mont_mul(u, pk[o], c.q, c.qneg_inv);
    c0 = add_mod(add_mod(c0, e1h[o], c.q), mh[o], c.q);
    uint32_t c1 = add_mod(mont_mul(u, pk[P1 + o], c.q, c.qneg_inv), e2h[o], c.q);
    ct[o] = c0;
    ct[P1 + o] = c1;
}

// x_j = c0 + c1 s (+ c2 s^2) per limb (NTT domain)
// grid (N/256, L, messages): ciphertext z (size * L * N words apart) into
// x + z * L * N
__global__ void dec_phase_kernel(const uint32_t *__restrict__ ct, uint32_t size, const uint32_t *__restrict__ sk,
                                 uint32_t *__restrict__ x, uint32_t N, uint32_t L,
                                 const ModConst *__restrict__ mcs) {
    const uint32_t j = blockIdx.y, k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const ModConst c = mcs[j];
    const size_t o = (size_t)j * N + k, P1 = (size_t)L * N;
    ct += blockIdx.z * size * P1;
    x += blockIdx.z * P1;
    const uint32_t s = sk[o];
    uint32_t v = add_mod(ct[o], mulmod_plain(ct[P1 + o], s, c), c.q);
    if (size == 3) v = add_mod(v, mulmod_plain(ct[2 * P1 + o], mulmod_plain(s, s, c), c), c.q);
    x[o] = v;
}

// m = round(t x / Q) mod t from the coefficient residues of x, exactly.
// grid (N/256, messages): x + y * L * N (coefficient form) into pt + y * N
__global__ void dec_round_kernel(const uint32_t *__restrict__ x, uint32_t *__restrict__ pt, uint32_t N,
                                 const ModConst *__restrict__ mcs, const MrcConst *__restrict__ mrc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int L = (int)mrc->L;
    x += (size_t)blockIdx.y * L * N;
    pt += (size_t)blockIdx.y * N;
    const uint32_t t = mrc->t;
    uint32_t r[MAXL], v[MAXL];
#pragma unroll
    for (int i = 0; i < MAXL; ++i)
        r[i] = i < L ? shoup(x[(size_t)i * N + k], mrc->tq[i], mrc->tqp[i], mcs[i].q) : 0;
    mrc_digits<MAXL>(r, v, L, mcs, mrc->invQ, mrc->invQp);       // digits of R = t x mod Q
    const uint32_t Rt = mrc_eval<MAXL>(v, L, mrc->wQt, mrc->wQtp, t);
    const bool carry = mrc_greater<MAXL>(v, L, mrc->hQ);
    // floor(t x / Q) = (t x - R) / Q = -R Q^-1 (mod t)
    uint32_t m = shoup(sub_mod(0, Rt, t), mrc->Qinvt, mrc->Qinvtp, t);
    if (carry) m = add_mod(m, 1, t);
    pt[k] = m;
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_set_key_words(lola_ctx *ctx, const uint32_t *words_host) {
    if (!ctx) return set_error(LOLA_E_INVAL, "null argument");
    for (int k = 0; k < 6; ++k) ctx->key_hi[k] = words_host ? words_host[k] : 0u;
    return LOLA_OK;
}

int lola_keygen_secret(lola_ctx *ctx, uint64_t seed, uint32_t *sk, lola_stream stream) {
    if (!ctx || !sk) return set_error(LOLA_E_INVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    void *buf = nullptr;
    int rc = scratch_get(ctx, (size_t)ctx->N * 4, &buf);
    if (rc) return rc;
    rc = launch_samples(ctx, seed, {SampleJob{(uint32_t *)buf, DOM_SK, 0, 0, SAMPLE_TERNARY, 0, 0}}, s);
    if (rc) return rc;
    std::vector<NttJob> jobs;
    for (uint32_t j = 0; j < ctx->L + ctx->K; ++j)
        jobs.push_back(NttJob{(const uint32_t *)buf, sk + (size_t)j * ctx->N, j, NTT_SRC_SIGNED32});
    return launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), s);
}

int lola_keygen_public(lola_ctx *ctx, uint64_t seed, const uint32_t *sk, uint32_t *pk, lola_stream stream) {
    if (!ctx || !sk || !pk) return set_error(LOLA_E_INVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = ctx->N, L = ctx->L;
    void *buf = nullptr;
    int rc = scratch_get(ctx, (1 + 2 * L) * N * 4 + L * N * 4, &buf);
    if (rc) return rc;
    uint32_t *E = (uint32_t *)buf, *A = E + N, *Ah = A + L * N, *Eh = Ah + L * N;
    std::vector<SampleJob> sj{SampleJob{E, DOM_PK_E, 0, 0, SAMPLE_CBD, 0, 0}};
    for (uint32_t j = 0; j < L; ++j)
        sj.push_back(SampleJob{A + j * N, DOM_PK_A, 0, j, SAMPLE_UNIFORM, ctx->primes[j], 0});
    if ((rc = launch_samples(ctx, seed, sj, s))) return rc;
    std::vector<NttJob> jobs;
    for (uint32_t j = 0; j < L; ++j) {
        jobs.push_back(NttJob{A + j * N, Ah + j * N, j, 0});
        jobs.push_back(NttJob{E, Eh + j * N, j, NTT_SRC_SIGNED32});
    }
    if ((rc = launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), s))) return rc;
    hipLaunchKernelGGL(pk_combine_kernel, dim3((unsigned)(N / 256), (unsigned)L), dim3(256), 0, s, Ah, Eh, sk, pk,
                       (uint32_t)N, (uint32_t)L, ctx->d_mc);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int lola_keygen_switch(lola_ctx *ctx, uint64_t seed, const uint32_t *sk, uint32_t galois, uint32_t *ksk,
                       lola_stream stream) {
    if (!ctx || !sk || !ksk) return set_error(LOLA_E_INVAL, "null argument");
    if (galois != 0 && (!(galois & 1) || galois >= 2 * ctx->N)) return set_error(LOLA_E_INVAL, "bad Galois element");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = ctx->N, L = ctx->L, M = L + ctx->K, DN = ctx->dnum();
    void *buf = nullptr;
    // s' [M][N], per digit: e [N] + a [M][N] raw, then transformed ahat/ehat [dn][M][N] each
    const size_t words = M * N + DN * (N + M * N) + 2 * DN * M * N;
    int rc = scratch_get(ctx, words * 4, &buf);
    if (rc) return rc;
    uint32_t *Sp = (uint32_t *)buf, *E = Sp + M * N, *A = E + DN * N, *Ah = A + DN * M * N, *Eh = Ah + DN * M * N;
    hipLaunchKernelGGL(sprime_kernel, dim3((unsigned)(N / 256), (unsigned)M), dim3(256), 0, s, sk, Sp,
                       (uint32_t)N, ctx->logN, galois, ctx->d_mc);
    LOLA_HIP(hipGetLastError());
    std::vector<SampleJob> sj;
    std::vector<NttJob> jobs;
    for (uint32_t i = 0; i < DN; ++i) {
        const uint32_t obj = (galois << 8) | i;
        sj.push_back(SampleJob{E + i * N, DOM_KSK_E, obj, 0, SAMPLE_CBD, 0, 0});
        for (uint32_t j = 0; j < M; ++j) {
            sj.push_back(SampleJob{A + (i * M + j) * N, DOM_KSK_A, obj, j, SAMPLE_UNIFORM, ctx->primes[j], 0});
            jobs.push_back(NttJob{A + (i * M + j) * N, Ah + (i * M + j) * N, j, 0});
            jobs.push_back(NttJob{E + i * N, Eh + (i * M + j) * N, j, NTT_SRC_SIGNED32});
        }
    }
    if ((rc = launch_samples(ctx, seed, sj, s))) return rc;
    if ((rc = launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), s))) return rc;
    hipLaunchKernelGGL(ksk_combine_kernel, dim3((unsigned)(N / 256), (unsigned)M, (unsigned)DN), dim3(256), 0, s,
                       Ah, Eh, sk, Sp, ksk, (uint32_t)N, (uint32_t)L, ctx->K, ctx->d_mc, ctx->d_mrc);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int lola_encrypt_batch(lola_ctx *ctx, const uint32_t *pk, const uint32_t *pt, uint32_t n, uint64_t seed,
                       uint32_t nonce0, uint32_t *ct, lola_stream stream) {
    if (!ctx || !pk || (n && (!pt || !ct))) return set_error(LOLA_E_INVAL, "null argument");
    if ((uint64_t)nonce0 + n > (1ull << 32)) return set_error(LOLA_E_INVAL, "nonce0 + n exceeds 2^32");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = ctx->N, L = ctx->L, W = 3 * N + 4 * L * N;   // scratch words per message
    for (uint32_t m0 = 0; m0 < n; m0 += CLIENT_CHUNK) {
        const uint32_t c = std::min(CLIENT_CHUNK, n - m0);
        void *buf = nullptr;
        int rc = scratch_get(ctx, c * W * 4, &buf);
        if (rc) return rc;
        std::vector<SampleJob> sj;
        std::vector<NttJob> jobs;
        for (uint32_t m = 0; m < c; ++m) {
            uint32_t *U = (uint32_t *)buf + m * W, *E1 = U + N, *E2 = E1 + N, *Uh = E2 + N, *E1h = Uh + L * N,
                     *E2h = E1h + L * N, *Mh = E2h + L * N;
            const uint32_t nonce = nonce0 + m0 + m;
            sj.push_back(SampleJob{U, DOM_ENC_U, nonce, 0, SAMPLE_TERNARY, 0, 0});
            sj.push_back(SampleJob{E1, DOM_ENC_E1, nonce, 0, SAMPLE_CBD, 0, 0});
            sj.push_back(SampleJob{E2, DOM_ENC_E2, nonce, 0, SAMPLE_CBD, 0, 0});
            for (uint32_t j = 0; j < L; ++j) {
                jobs.push_back(NttJob{U, Uh + j * N, j, NTT_SRC_SIGNED32});
                jobs.push_back(NttJob{E1, E1h + j * N, j, NTT_SRC_SIGNED32});
                jobs.push_back(NttJob{E2, E2h + j * N, j, NTT_SRC_SIGNED32});
                jobs.push_back(NttJob{pt + (m0 + m) * N, Mh + j * N, j, NTT_MUL_DELTA});
            }
        }
        if ((rc = launch_samples(ctx, seed, sj, s))) return rc;
        if ((rc = launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), s))) return rc;
        const uint32_t *Uh = (const uint32_t *)buf + 3 * N;
        hipLaunchKernelGGL(enc_combine_kernel, dim3((unsigned)(N / 256), (unsigned)L, c), dim3(256), 0, s, pk, Uh,
                           Uh + L * N, Uh + 2 * L * N, Uh + 3 * L * N, W, ct + m0 * 2 * L * N, (uint32_t)N,
                           (uint32_t)L, ctx->d_mc);
        LOLA_HIP(hipGetLastError());
    }
    return LOLA_OK;
}

int lola_encrypt(lola_ctx *ctx, const uint32_t *pk, const uint32_t *pt, uint64_t seed, uint32_t nonce,
                 uint32_t *ct, lola_stream stream) {
    if (!ctx || !pk || !pt || !ct) return set_error(LOLA_E_INVAL, "null argument");
    return lola_encrypt_batch(ctx, pk, pt, 1, seed, nonce, ct, stream);
}

int lola_decrypt_batch(lola_ctx *ctx, const uint32_t *sk, const uint32_t *ct, uint32_t n, uint32_t size,
                       uint32_t *pt, lola_stream stream) {
    if (!ctx || !sk || (n && (!ct || !pt))) return set_error(LOLA_E_INVAL, "null argument");
    if (size != 2 && size != 3) return set_error(LOLA_E_SHAPE, "ciphertext size must be 2 or 3");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = ctx->N, L = ctx->L;
    for (uint32_t m0 = 0; m0 < n; m0 += CLIENT_CHUNK) {
        const uint32_t c = std::min(CLIENT_CHUNK, n - m0);
        void *buf = nullptr;
        int rc = scratch_get(ctx, 2 * c * L * N * 4, &buf);
        if (rc) return rc;
        uint32_t *X = (uint32_t *)buf, *Xc = X + c * L * N;
        hipLaunchKernelGGL(dec_phase_kernel, dim3((unsigned)(N / 256), (unsigned)L, c), dim3(256), 0, s,
                           ct + m0 * size * L * N, size, sk, X, (uint32_t)N, (uint32_t)L, ctx->d_mc);
        LOLA_HIP(hipGetLastError());
        std::vector<NttJob> jobs;
        for (uint32_t m = 0; m < c; ++m)
            for (uint32_t j = 0; j < L; ++j)
                jobs.push_back(NttJob{X + (m * L + j) * N, Xc + (m * L + j) * N, j, NTT_INVERSE});
        if ((rc = launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), s))) return rc;
        hipLaunchKernelGGL(dec_round_kernel, dim3((unsigned)(N / 256), c), dim3(256), 0, s, Xc, pt + m0 * N,
                           (uint32_t)N, ctx->d_mc, ctx->d_mrc);
        LOLA_HIP(hipGetLastError());
    }
    return LOLA_OK;
}

int lola_decrypt(lola_ctx *ctx, const uint32_t *sk, const uint32_t *ct, uint32_t size, uint32_t *pt,
                 lola_stream stream) {
    if (!ctx || !sk || !ct || !pt) return set_error(LOLA_E_INVAL, "null argument");
    return lola_decrypt_batch(ctx, sk, ct, 1, size, pt, stream);
}

int lola_export_sk(lola_ctx *ctx, const uint32_t *sk, uint32_t *out, lola_stream stream) {
    if (!ctx || !sk || !out) return set_error(LOLA_E_INVAL, "null argument");
    std::vector<NttJob> jobs;
    for (uint32_t j = 0; j < ctx->L + ctx->K; ++j)
        jobs.push_back(NttJob{sk + (size_t)j * ctx->N, out + (size_t)j * ctx->N, j, NTT_INVERSE});
    return launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), (hipStream_t)stream);
}

int lola_export_pk(lola_ctx *ctx, const uint32_t *pk, uint32_t *out, lola_stream stream) {
    if (!ctx || !pk || !out) return set_error(LOLA_E_INVAL, "null argument");
    std::vector<NttJob> jobs;
    for (uint32_t c = 0; c < 2; ++c)
        for (uint32_t j = 0; j < ctx->L; ++j) {
            size_t o = ((size_t)c * ctx->L + j) * ctx->N;
            jobs.push_back(NttJob{pk + o, out + o, j, NTT_INVERSE | NTT_FROM_MONT});
        }
    return launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), (hipStream_t)stream);
}

int lola_export_ksk(lola_ctx *ctx, const uint32_t *ksk, uint32_t *out, lola_stream stream) {
    if (!ctx || !ksk || !out) return set_error(LOLA_E_INVAL, "null argument");
    std::vector<NttJob> jobs;
    const uint32_t M = ctx->L + ctx->K;
    for (uint32_t i = 0; i < ctx->dnum(); ++i)
        for (uint32_t c = 0; c < 2; ++c)
            for (uint32_t j = 0; j < M; ++j) {
                size_t o = (((size_t)i * 2 + c) * M + j) * ctx->N;
                jobs.push_back(NttJob{ksk + o, out + o, j, NTT_INVERSE | NTT_FROM_MONT});
            }
    return launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), (hipStream_t)stream);
}

}  // extern "C"
