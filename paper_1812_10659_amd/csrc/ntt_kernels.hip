// Batched limb NTTs: one workgroup per (limb, prime) job.
#include "lola_internal.hpp"
#include "ntt_core.hpp"

namespace lola {

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ntt_jobs_kernel(
    const NttJob *__restrict__ jobs, const ModConst *__restrict__ mcs, const TwPair *__restrict__ tw,
    const TwPair *__restrict__ itw, uint32_t t, const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[1 << LOGN];
    const NttJob job = jobs[blockIdx.x];
    const ModConst mc = mcs[job.prime];
    const uint32_t tid = threadIdx.x;
    const size_t toff = (size_t)job.prime << LOGN;
    constexpr uint32_t N = 1u << LOGN;
    const GBuf src = gbuf(job.src, N), dst = gbuf(job.dst, N);
    uint32_t x[NTT_E];
    if (!(job.flags & NTT_INVERSE)) {
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) {
            uint32_t v = gld(src, natural_index<LOGN>(tid, r));
            if (job.flags & NTT_SRC_SIGNED_T) {
                // [v]_t mod q: values above t/2 stand for v - t
                v = (v > (t >> 1)) ? mc.q - (t - v) : v;
            }
            if (job.flags & NTT_SRC_SIGNED32) {
                const int32_t sv = (int32_t)v;
                v = sv < 0 ? mc.q - (uint32_t)(-sv) : (uint32_t)sv;
            }
            if (job.flags & NTT_SRC_REDUCE) v = reduce32(v, mc.q, mc.one_shoup);
            x[r] = v;
        }
        ntt_fwd_regs<LOGN>(x, tid, sh, tw + toff, mc.q);
        if (job.flags & NTT_MUL_DELTA) {
            const uint32_t d = mrc->deltaq[job.prime], dp = mrc->deltaqp[job.prime];
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) x[r] = shoup(x[r], d, dp, mc.q);
        }
        if (job.flags & NTT_TO_MONT) {
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) x[r] = shoup(x[r], mc.r_mod, mc.r_shoup, mc.q);
        }
        store_spectral<LOGN>(dst, tid, x);
    } else {
        load_spectral<LOGN>(src, tid, x);
        if (job.flags & NTT_FROM_MONT) {
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) x[r] = mont_mul(x[r], 1u, mc.q, mc.qneg_inv);
        }
        ntt_inv_regs<LOGN>(x, tid, sh, itw + toff, mc);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(dst, natural_index<LOGN>(tid, r), x[r]);
    }
}

int launch_ntt_jobs_dev(lola_ctx *ctx, const NttJob *d_jobs, int n, hipStream_t s) {
    if (n <= 0) return LOLA_OK;
    const dim3 grid(n), block(ctx->N / NTT_E);
#define LOLA_NTT_CASE(LG)                                                                              \
    case LG:                                                                                           \
        hipLaunchKernelGGL(ntt_jobs_kernel<LG>, grid, block, 0, s, d_jobs, ctx->d_mc, ctx->d_tw,      \
                           ctx->d_itw, ctx->t, ctx->d_mrc);                                             \
        break;
    switch (ctx->logN) {
        LOLA_NTT_CASE(10)
        LOLA_NTT_CASE(11)
        LOLA_NTT_CASE(12)
        LOLA_NTT_CASE(13)
        LOLA_NTT_CASE(14)
        default: return set_error(LOLA_E_PARAMS, "unsupported N");
    }
#undef LOLA_NTT_CASE
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int launch_ntt_jobs(lola_ctx *ctx, const NttJob *host_jobs, int n, hipStream_t s) {
    const int chunk = (int)(lola_ctx::RING_SLAB / sizeof(NttJob));
    for (int off = 0; off < n; off += chunk) {
        int m = std::min(chunk, n - off);
        void *d = nullptr;
        int rc = desc_upload(ctx, host_jobs + off, m * sizeof(NttJob), s, &d);
        if (rc) return rc;
        rc = launch_ntt_jobs_dev(ctx, (const NttJob *)d, m, s);
        if (rc) return rc;
    }
    return LOLA_OK;
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_ntt_limbs(lola_ctx *ctx, const uint32_t *in_dev, uint32_t *out_dev, uint32_t n_limbs,
                   const uint32_t *prime_idx_host, int inverse, lola_stream stream) {
    if (!ctx || !in_dev || !out_dev || !prime_idx_host) return set_error(LOLA_E_INVAL, "null argument");
    std::vector<NttJob> jobs(n_limbs);
    for (uint32_t k = 0; k < n_limbs; ++k) {
        if (prime_idx_host[k] >= ctx->nprimes()) return set_error(LOLA_E_INVAL, "prime index out of range");
        jobs[k] = NttJob{in_dev + (size_t)k * ctx->N, out_dev + (size_t)k * ctx->N, prime_idx_host[k],
                         inverse ? NTT_INVERSE : 0u};
    }
    return launch_ntt_jobs(ctx, jobs.data(), (int)n_limbs, (hipStream_t)stream);
}

int lola_to_coeff(lola_ctx *ctx, const uint32_t *in_dev, uint32_t n_polys, uint32_t *out_dev,
                  lola_stream stream) {
    if (!ctx || !in_dev || !out_dev) return set_error(LOLA_E_INVAL, "null argument");
    std::vector<NttJob> jobs;
    for (uint32_t p = 0; p < n_polys; ++p)
        for (uint32_t i = 0; i < ctx->L; ++i) {
            size_t off = ((size_t)p * ctx->L + i) * ctx->N;
            jobs.push_back(NttJob{in_dev + off, out_dev + off, i, NTT_INVERSE});
        }
    return launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), (hipStream_t)stream);
}

int lola_from_coeff(lola_ctx *ctx, const uint32_t *in_dev, uint32_t n_polys, uint32_t *out_dev,
                    lola_stream stream) {
    if (!ctx || !in_dev || !out_dev) return set_error(LOLA_E_INVAL, "null argument");
    std::vector<NttJob> jobs;
    for (uint32_t p = 0; p < n_polys; ++p)
        for (uint32_t i = 0; i < ctx->L; ++i) {
            size_t off = ((size_t)p * ctx->L + i) * ctx->N;
            jobs.push_back(NttJob{in_dev + off, out_dev + off, i, NTT_SRC_REDUCE});
        }
    return launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), (hipStream_t)stream);
}

}  // extern "C"
