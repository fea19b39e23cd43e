// Element-wise ciphertext operations in the NTT domain, slot encoding and
// plaintext forms.  These are HBM-bound streams: each thread moves 4 words
// with 128-bit loads and stores; the limb of a word is (word / N) mod L.
#include <algorithm>
#include <vector>

#include "lola_internal.hpp"

namespace lola {

struct LimbScalars {            // per-limb constant with its Shoup companion
    uint32_t w[MAXL], wp[MAXL];
};

__global__ void ew_add_kernel(const uint4 *__restrict__ a, const uint4 *__restrict__ b, uint4 *__restrict__ out,
                              size_t n4, uint32_t logN, uint32_t L, const ModConst *__restrict__ mcs) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const uint32_t limb = (uint32_t)(((i * 4) >> logN) % L);
    const uint32_t q = mcs[limb].q;
    uint4 x = a[i], y = b[i];
    out[i] = make_uint4(add_mod(x.x, y.x, q), add_mod(x.y, y.y, q), add_mod(x.z, y.z, q), add_mod(x.w, y.w, q));
}

__global__ void ew_mul_scalar_kernel(const uint4 *__restrict__ a, uint4 *__restrict__ out, size_t n4,
                                     uint32_t logN, uint32_t L, const ModConst *__restrict__ mcs,
                                     LimbScalars ws) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const uint32_t limb = (uint32_t)(((i * 4) >> logN) % L);
    const uint32_t q = mcs[limb].q, w = ws.w[limb], wp = ws.wp[limb];
    uint4 x = a[i];
    out[i] = make_uint4(shoup(x.x, w, wp, q), shoup(x.y, w, wp, q), shoup(x.z, w, wp, q), shoup(x.w, w, wp, q));
}

// out[c][j][k] = ct[c][j][k] * pt[j][k], pt in Montgomery form.
__global__ void ew_mul_plain_kernel(const uint4 *__restrict__ ct, const uint4 *__restrict__ pt,
                                    uint4 *__restrict__ out, size_t n4, uint32_t logN, uint32_t L,
                                    const ModConst *__restrict__ mcs) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const size_t poly4 = ((size_t)L << logN) / 4;
    const uint32_t limb = (uint32_t)(((i * 4) >> logN) % L);
    const ModConst &c = mcs[limb];
    uint4 x = ct[i], y = pt[i % poly4];
    out[i] = make_uint4(mont_mul(x.x, y.x, c.q, c.qneg_inv), mont_mul(x.y, y.y, c.q, c.qneg_inv),
                        mont_mul(x.z, y.z, c.q, c.qneg_inv), mont_mul(x.w, y.w, c.q, c.qneg_inv));
}

// out0 = c0 + pt (add form), out1 = c1.
__global__ void ew_add_plain_kernel(const uint4 *__restrict__ ct, const uint4 *__restrict__ pt,
                                    uint4 *__restrict__ out, size_t n4, uint32_t logN, uint32_t L,
                                    const ModConst *__restrict__ mcs) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const size_t poly4 = ((size_t)L << logN) / 4;
    uint4 x = ct[i];
    if (i < poly4) {
        const uint32_t q = mcs[(uint32_t)((i * 4) >> logN)].q;
        uint4 y = pt[i];
        x = make_uint4(add_mod(x.x, y.x, q), add_mod(x.y, y.y, q), add_mod(x.z, y.z, q), add_mod(x.w, y.w, q));
    }
    out[i] = x;
}

// grid (N / 256, messages): message blockIdx.y at offset blockIdx.y * N
__global__ void encode_scatter_kernel(const int64_t *__restrict__ slots, const uint32_t *__restrict__ pos,
                                      uint32_t *__restrict__ buf, uint32_t N, uint32_t t) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const size_t m = (size_t)blockIdx.y * N;
    int64_t v = slots[m + s] % (int64_t)t;
    if (v < 0) v += t;
    buf[m + pos[s]] = (uint32_t)v;
}

__global__ void decode_gather_kernel(const uint32_t *__restrict__ buf, const uint32_t *__restrict__ pos,
                                     int64_t *__restrict__ slots, uint32_t N) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const size_t m = (size_t)blockIdx.y * N;
    slots[m + s] = (int64_t)buf[m + pos[s]];
}

constexpr uint32_t CODEC_CHUNK = 64;   // messages per scratch fill (256 KiB each at N = 16384)

static inline dim3 grid_for(size_t n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

}  // namespace lola

using namespace lola;

extern "C" {

int lola_add(lola_ctx *ctx, const uint32_t *a, const uint32_t *b, uint32_t size, uint32_t *out,
             lola_stream stream) {
    if (!ctx || !a || !b || !out) return set_error(LOLA_E_INVAL, "null argument");
    if (size < 1 || size > 3) return set_error(LOLA_E_SHAPE, "size must be 1, 2 or 3");
    size_t n4 = (size_t)size * ctx->L * ctx->N / 4;
    hipLaunchKernelGGL(ew_add_kernel, grid_for(n4, 256), dim3(256), 0, (hipStream_t)stream, (const uint4 *)a,
                       (const uint4 *)b, (uint4 *)out, n4, ctx->logN, ctx->L, ctx->d_mc);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int lola_mul_scalar(lola_ctx *ctx, const uint32_t *ct, int64_t w, uint32_t *out, lola_stream stream) {
    if (!ctx || !ct || !out) return set_error(LOLA_E_INVAL, "null argument");
    // [w]_t, then its residue mod every q_j
    int64_t wt = w % (int64_t)ctx->t;
    if (wt < 0) wt += ctx->t;
    if (wt > (int64_t)(ctx->t / 2)) wt -= ctx->t;
    LimbScalars ws{};
    for (uint32_t j = 0; j < ctx->L; ++j) {
        int64_t q = ctx->primes[j];
        int64_t r = wt % q;
        if (r < 0) r += q;
        ws.w[j] = (uint32_t)r;
        ws.wp[j] = shoup_companion((uint32_t)r, (uint32_t)q);
    }
    size_t n4 = (size_t)2 * ctx->L * ctx->N / 4;
    hipLaunchKernelGGL(ew_mul_scalar_kernel, grid_for(n4, 256), dim3(256), 0, (hipStream_t)stream,
                       (const uint4 *)ct, (uint4 *)out, n4, ctx->logN, ctx->L, ctx->d_mc, ws);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int lola_mul_plain(lola_ctx *ctx, const uint32_t *ct, const uint32_t *ptm, uint32_t *out, lola_stream stream) {
    if (!ctx || !ct || !ptm || !out) return set_error(LOLA_E_INVAL, "null argument");
    size_t n4 = (size_t)2 * ctx->L * ctx->N / 4;
    hipLaunchKernelGGL(ew_mul_plain_kernel, grid_for(n4, 256), dim3(256), 0, (hipStream_t)stream,
                       (const uint4 *)ct, (const uint4 *)ptm, (uint4 *)out, n4, ctx->logN, ctx->L, ctx->d_mc);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int lola_add_plain(lola_ctx *ctx, const uint32_t *ct, const uint32_t *pta, uint32_t *out, lola_stream stream) {
    if (!ctx || !ct || !pta || !out) return set_error(LOLA_E_INVAL, "null argument");
    size_t n4 = (size_t)2 * ctx->L * ctx->N / 4;
    hipLaunchKernelGGL(ew_add_plain_kernel, grid_for(n4, 256), dim3(256), 0, (hipStream_t)stream,
                       (const uint4 *)ct, (const uint4 *)pta, (uint4 *)out, n4, ctx->logN, ctx->L, ctx->d_mc);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int lola_encode_batch(lola_ctx *ctx, const int64_t *slots, uint32_t n, uint32_t *pt, lola_stream stream) {
    if (!ctx || (n && (!slots || !pt))) return set_error(LOLA_E_INVAL, "null argument");
    const size_t N = ctx->N;
    hipStream_t s = (hipStream_t)stream;
    for (uint32_t m0 = 0; m0 < n; m0 += CODEC_CHUNK) {
        const uint32_t c = std::min(CODEC_CHUNK, n - m0);
        void *buf = nullptr;
        int rc = scratch_get(ctx, c * N * 4, &buf);
        if (rc) return rc;
        hipLaunchKernelGGL(encode_scatter_kernel, dim3((unsigned)((N + 255) / 256), c), dim3(256), 0, s,
                           slots + m0 * N, ctx->d_slotpos, (uint32_t *)buf, ctx->N, ctx->t);
        LOLA_HIP(hipGetLastError());
        std::vector<NttJob> jobs(c);
        for (uint32_t m = 0; m < c; ++m)
            jobs[m] = NttJob{(const uint32_t *)buf + m * N, pt + (m0 + m) * N, ctx->idxT(), NTT_INVERSE};
        if ((rc = launch_ntt_jobs(ctx, jobs.data(), (int)c, s))) return rc;
    }
    return LOLA_OK;
}

int lola_decode_batch(lola_ctx *ctx, const uint32_t *pt, uint32_t n, int64_t *slots, lola_stream stream) {
    if (!ctx || (n && (!slots || !pt))) return set_error(LOLA_E_INVAL, "null argument");
    const size_t N = ctx->N;
    hipStream_t s = (hipStream_t)stream;
    for (uint32_t m0 = 0; m0 < n; m0 += CODEC_CHUNK) {
        const uint32_t c = std::min(CODEC_CHUNK, n - m0);
        void *buf = nullptr;
        int rc = scratch_get(ctx, c * N * 4, &buf);
        if (rc) return rc;
        std::vector<NttJob> jobs(c);
        for (uint32_t m = 0; m < c; ++m)
            jobs[m] = NttJob{pt + (m0 + m) * N, (uint32_t *)buf + m * N, ctx->idxT(), NTT_SRC_REDUCE};
        if ((rc = launch_ntt_jobs(ctx, jobs.data(), (int)c, s))) return rc;
        hipLaunchKernelGGL(decode_gather_kernel, dim3((unsigned)((N + 255) / 256), c), dim3(256), 0, s,
                           (const uint32_t *)buf, ctx->d_slotpos, slots + m0 * N, ctx->N);
        LOLA_HIP(hipGetLastError());
    }
    return LOLA_OK;
}

int lola_encode(lola_ctx *ctx, const int64_t *slots, uint32_t *pt, lola_stream stream) {
    if (!ctx || !slots || !pt) return set_error(LOLA_E_INVAL, "null argument");
    return lola_encode_batch(ctx, slots, 1, pt, stream);
}

int lola_decode(lola_ctx *ctx, const uint32_t *pt, int64_t *slots, lola_stream stream) {
    if (!ctx || !slots || !pt) return set_error(LOLA_E_INVAL, "null argument");
    return lola_decode_batch(ctx, pt, 1, slots, stream);
}

int lola_plain_mul_form(lola_ctx *ctx, const uint32_t *pt, uint32_t *out, lola_stream stream) {
    if (!ctx || !pt || !out) return set_error(LOLA_E_INVAL, "null argument");
    std::vector<NttJob> jobs(ctx->L);
    for (uint32_t j = 0; j < ctx->L; ++j)
        jobs[j] = NttJob{pt, out + (size_t)j * ctx->N, j, NTT_SRC_SIGNED_T | NTT_TO_MONT};
    return launch_ntt_jobs(ctx, jobs.data(), (int)ctx->L, (hipStream_t)stream);
}

int lola_plain_add_form(lola_ctx *ctx, const uint32_t *pt, uint32_t *out, lola_stream stream) {
    if (!ctx || !pt || !out) return set_error(LOLA_E_INVAL, "null argument");
    std::vector<NttJob> jobs(ctx->L);
    for (uint32_t j = 0; j < ctx->L; ++j) jobs[j] = NttJob{pt, out + (size_t)j * ctx->N, j, NTT_MUL_DELTA};
    return launch_ntt_jobs(ctx, jobs.data(), (int)ctx->L, (hipStream_t)stream);
}

}  // extern "C"
