// Batched element-wise jobs, the program runner, and kernel timing.
#include "program.hpp"

namespace lola {

// dst = sum_k w_k src_k (+ add on component 0).  grid (2LN/4/256, jobs)
//
// A block's 1024 words lie in one limb (N >= 1024), so the limb and the
// weights are uniform and come from scalar loads.  Sources are taken in
// groups of LIN_GROUP with all their loads issued before any product: a
// group past the last source repeats the last source's address with weight
// 0 (a zero term), which keeps the group one straight block instead of a
// test and a wait per source.
constexpr uint32_t LIN_GROUP = 8;

__global__ void lin_kernel(const LinJob *__restrict__ jobs, uint32_t logN, uint32_t L,
                           const ModConst *__restrict__ mcs) {
    const LinJob &job = jobs[blockIdx.y];
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n4 = ((size_t)2 * L << logN) / 4;
    if (i >= n4) return;
    const uint32_t cl = (uint32_t)(((size_t)blockIdx.x * blockDim.x * 4) >> logN);   // component * L + limb
    const uint32_t limb = cl % L;
    const uint32_t q = mcs[limb].q;
    const uint32_t n = job.n_src;
    uint4 acc = make_uint4(0, 0, 0, 0);
    for (uint32_t k0 = 0; k0 < n; k0 += LIN_GROUP) {
        uint4 x[LIN_GROUP];
#pragma unroll
        for (uint32_t b = 0; b < LIN_GROUP; ++b) x[b] = ((const uint4 *)job.srcs[min(k0 + b, n - 1)])[i];
#pragma unroll
        for (uint32_t b = 0; b < LIN_GROUP; ++b) {
            // weights of the clamped source, masked to 0 past the last one
            const uint32_t k = min(k0 + b, n - 1), mask = 0u - (uint32_t)(k0 + b < n);
            const uint32_t w = job.w[(2 * k) * L + limb] & mask, wp = job.w[(2 * k + 1) * L + limb] & mask;
            acc.x = add_mod(acc.x, shoup(x[b].x, w, wp, q), q);
            acc.y = add_mod(acc.y, shoup(x[b].y, w, wp, q), q);
            acc.z = add_mod(acc.z, shoup(x[b].z, w, wp, q), q);
            acc.w = add_mod(acc.w, shoup(x[b].w, w, wp, q), q);
        }
    }
    if (job.add && cl < L) {
        const uint4 y = ((const uint4 *)job.add)[i];
        acc = make_uint4(add_mod(acc.x, y.x, q), add_mod(acc.y, y.y, q), add_mod(acc.z, y.z, q),
                         add_mod(acc.w, y.w, q));
    }
    ((uint4 *)job.dst)[i] = acc;
}

// dst = src * mul (+ add on component 0).  grid (2LN/4/256, jobs)
__global__ void plain_kernel(const PlainJob *__restrict__ jobs, uint32_t logN, uint32_t L,
                             const ModConst *__restrict__ mcs) {
    const PlainJob job = jobs[blockIdx.y];
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t poly4 = ((size_t)L << logN) / 4;
    if (i >= 2 * poly4) return;
    const uint32_t cl = (uint32_t)((i * 4) >> logN);
    const ModConst &c = mcs[cl % L];
    uint4 x = ((const uint4 *)job.src)[i];
    if (job.mul) {
        const uint4 y = ((const uint4 *)job.mul)[i % poly4];
        x = make_uint4(mont_mul(x.x, y.x, c.q, c.qneg_inv), mont_mul(x.y, y.y, c.q, c.qneg_inv),
                       mont_mul(x.z, y.z, c.q, c.qneg_inv), mont_mul(x.w, y.w, c.q, c.qneg_inv));
    }
    if (job.add && i < poly4) {
        const uint4 y = ((const uint4 *)job.add)[i];
        x = make_uint4(add_mod(x.x, y.x, c.q), add_mod(x.y, y.y, c.q), add_mod(x.z, y.z, c.q),
                       add_mod(x.w, y.w, c.q));
    }
    ((uint4 *)job.dst)[i] = x;
}

int launch_lin_dev(lola_ctx *ctx, const LinJob *d, uint32_t n, hipStream_t s) {
    const size_t n4 = (size_t)2 * ctx->L * ctx->N / 4;
    hipLaunchKernelGGL(lin_kernel, dim3((unsigned)((n4 + 255) / 256), n), dim3(256), 0, s, d, ctx->logN, ctx->L,
                       ctx->d_mc);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int launch_plain_dev(lola_ctx *ctx, const PlainJob *d, uint32_t n, hipStream_t s) {
    const size_t n4 = (size_t)2 * ctx->L * ctx->N / 4;
    hipLaunchKernelGGL(plain_kernel, dim3((unsigned)((n4 + 255) / 256), n), dim3(256), 0, s, d, ctx->logN,
                       ctx->L, ctx->d_mc);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int program_run_launch(lola_ctx *ctx, const Launch &l, const uint8_t *d_blob, hipStream_t s) {
    const void *d = d_blob + l.off;
    switch (l.kind) {
        case LK_NTT: return launch_ntt_jobs_dev(ctx, (const NttJob *)d, (int)l.n, s);
        case LK_LIN: return launch_lin_dev(ctx, (const LinJob *)d, l.n, s);
        case LK_PLAIN: return launch_plain_dev(ctx, (const PlainJob *)d, l.n, s);
        case LK_KS: return launch_keyswitch(ctx, (const KsJob *)d, l.n, s);
        case LK_KS_HSRC: return launch_keyswitch_hoist_src(ctx, (const KsJob *)d, l.n, s);
        case LK_KS_HROT: return launch_keyswitch_hoist_rot(ctx, (const KsJob *)d, l.n, s);
        case LK_MUL_EXTEND:
        case LK_MUL_PRODUCT:
        case LK_MUL_ROUND: return launch_mul_stage(ctx, l.kind, (const MulJob *)d, l.n, s);
        default: return set_error(LOLA_E_INVAL, "bad launch kind");
    }
}

int program_run(lola_ctx *ctx, const Program &p, const uint8_t *d_blob, hipStream_t s) {
    for (const Launch &l : p.launches) {
        int rc = program_run_launch(ctx, l, d_blob, s);
        if (rc) return rc;
    }
    return LOLA_OK;
}

int program_run_now(lola_ctx *ctx, const Program &p, hipStream_t s) {
    if (p.launches.empty()) return LOLA_OK;
    void *d = nullptr;
    int rc = desc_upload(ctx, p.blob.data(), p.blob.size(), s, &d);
    if (rc) return rc;
    return program_run(ctx, p, (const uint8_t *)d, s);
}

int timing_pair(lola_ctx *ctx, hipEvent_t *a, hipEvent_t *b) {
    for (int k = 0; k < 2; ++k) {
        if (ctx->timing_pool.empty()) {
            hipEvent_t e;
            LOLA_HIP(hipEventCreate(&e));
            ctx->timing_pool.push_back(e);
        }
        hipEvent_t e = ctx->timing_pool.back();
        ctx->timing_pool.pop_back();
        ctx->timing_events.push_back(e);
        (k == 0 ? *a : *b) = e;
    }
    return LOLA_OK;
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_timing_enable(lola_ctx *ctx, int on) {
    if (!ctx) return set_error(LOLA_E_INVAL, "null argument");
    ctx->timing = on != 0;
    return LOLA_OK;
}

int lola_kernel_timing(lola_ctx *ctx, double *total_ms, uint64_t *launches, uint64_t *jobs) {
    if (!ctx || !total_ms || !launches || !jobs) return set_error(LOLA_E_INVAL, "null argument");
    double tot = 0;
    const size_t npairs = ctx->timing_events.size() / 2;
    for (size_t k = 0; k < npairs; ++k) {
        hipEvent_t a = ctx->timing_events[2 * k], b = ctx->timing_events[2 * k + 1];
        LOLA_HIP(hipEventSynchronize(b));
        float ms = 0;
        LOLA_HIP(hipEventElapsedTime(&ms, a, b));
        tot += ms;
    }
    *total_ms = tot;
    *launches = npairs;
    *jobs = ctx->timed_jobs;
    for (hipEvent_t e : ctx->timing_events) ctx->timing_pool.push_back(e);
    ctx->timing_events.clear();
    ctx->timed_jobs = 0;
    return LOLA_OK;
}

}  // extern "C"

extern "C" {

int lola_mul_plain_batch(lola_ctx *ctx, uint32_t n, const uint32_t *const *ct, const uint32_t *const *pt,
                         uint32_t *const *out, lola_stream stream) {
    if (!ctx || (n && (!ct || !pt || !out))) return set_error(LOLA_E_INVAL, "null argument");
    const uint32_t chunk = (uint32_t)(lola_ctx::RING_SLAB / sizeof(PlainJob) / 2);
    for (uint32_t off = 0; off < n; off += chunk) {
        const uint32_t m = std::min(chunk, n - off);
        Program p;
        std::vector<PlainJob> jobs(m);
        for (uint32_t k = 0; k < m; ++k) {
            if (!ct[off + k] || !pt[off + k] || !out[off + k]) return set_error(LOLA_E_INVAL, "null pointer in batch");
            jobs[k] = PlainJob{ct[off + k], pt[off + k], nullptr, out[off + k]};
        }
        p.launch(LK_PLAIN, jobs);
        int rc = program_run_now(ctx, p, (hipStream_t)stream);
        if (rc) return rc;
    }
    return LOLA_OK;
}

int lola_mul_batch(lola_ctx *ctx, uint32_t n, const uint32_t *const *a, const uint32_t *const *b,
                   uint32_t *const *out3, lola_stream stream) {
    if (!ctx || (n && (!a || !b || !out3))) return set_error(LOLA_E_INVAL, "null argument");
    return mul_batch(ctx, n, a, b, out3, (hipStream_t)stream);
}

}  // extern "C"
