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

// Cost: the launch's distinct sources and constants are read once (2LN and
// LN words), every job writes its ciphertext; each source word of each job
// takes a Shoup product and an add, each constant word an add.
int launch_lin_dev(lola_ctx *ctx, const LinJob *d, uint32_t n, const uint64_t *aux, hipStream_t s) {
    const size_t n4 = (size_t)2 * ctx->L * ctx->N / 4;
    const double ln = (double)ctx->L * ctx->N;
    LOLA_TIMED(ctx, s, KID_LIN, n, 4 * ln * (2.0 * (aux[1] + n) + aux[3]),
               ln * (2.0 * aux[0] * (COST_MUL + COST_ADD) + aux[2] * COST_ADD),
               hipLaunchKernelGGL(lin_kernel, dim3((unsigned)((n4 + 255) / 256), n), dim3(256), 0, s, d, ctx->logN,
                                  ctx->L, ctx->d_mc));
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

// Cost: every job reads and writes one ciphertext; the launch's distinct
// product and add constants (LN words) are read once; a product is a
// Montgomery product per word of both components, an add one per word of
// component 0.
int launch_plain_dev(lola_ctx *ctx, const PlainJob *d, uint32_t n, const uint64_t *aux, hipStream_t s) {
    const size_t n4 = (size_t)2 * ctx->L * ctx->N / 4;
    const double ln = (double)ctx->L * ctx->N;
    LOLA_TIMED(ctx, s, KID_PLAIN, n, 4 * ln * (4.0 * n + aux[1] + aux[3]),
               ln * (2.0 * aux[0] * COST_MUL + aux[2] * COST_ADD),
               hipLaunchKernelGGL(plain_kernel, dim3((unsigned)((n4 + 255) / 256), n), dim3(256), 0, s, d,
                                  ctx->logN, ctx->L, ctx->d_mc));
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int program_run_launch(lola_ctx *ctx, const Launch &l, const uint8_t *d_blob, hipStream_t s) {
    const void *d = d_blob + l.off;
    switch (l.kind) {
        case LK_NTT: return launch_ntt_jobs_dev(ctx, (const NttJob *)d, (int)l.n, s);
        case LK_LIN: return launch_lin_dev(ctx, (const LinJob *)d, l.n, l.aux, s);
        case LK_PLAIN: return launch_plain_dev(ctx, (const PlainJob *)d, l.n, l.aux, s);
        case LK_KS: return launch_keyswitch(ctx, (const KsJob *)d, l.n, l.aux, s);
        case LK_KS_HSRC: return launch_keyswitch_hoist_src(ctx, (const KsJob *)d, l.n, s);
        case LK_KS_HROT: return launch_keyswitch_hoist_rot(ctx, (const KsJob *)d, l.n, l.aux, s);
        case LK_MUL_EXTEND:
        case LK_MUL_PRODUCT:
        case LK_MUL_ROUND: return launch_mul_stage(ctx, l.kind, (const MulJob *)d, l.n, l.aux[0], s);
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

static int pool_event(lola_ctx *ctx, hipEvent_t *e) {
    if (ctx->timing_pool.empty()) {
        hipEvent_t x;
        LOLA_HIP(hipEventCreate(&x));
        ctx->timing_pool.push_back(x);
    }
    *e = ctx->timing_pool.back();
    ctx->timing_pool.pop_back();
    return LOLA_OK;
}

int ktime_begin(lola_ctx *ctx, hipStream_t s, hipEvent_t *a) {
    *a = nullptr;
    if (!ctx->timing) return LOLA_OK;
    hipEvent_t e;
    int rc = pool_event(ctx, &e);
    if (rc) return rc;
    if (hipEventRecord(e, s) != hipSuccess) {
        ctx->timing_pool.push_back(e);
        return set_error(LOLA_E_DEVICE, "timing event");
    }
    *a = e;
    return LOLA_OK;
}

int ktime_end(lola_ctx *ctx, hipStream_t s, hipEvent_t a, uint32_t kid, uint64_t units, double bytes, double ops) {
    hipEvent_t b;
    int rc = pool_event(ctx, &b);
    if (rc) {
        ctx->timing_pool.push_back(a);
        return rc;
    }
    if (hipEventRecord(b, s) != hipSuccess) {
        ctx->timing_pool.push_back(a);
        ctx->timing_pool.push_back(b);
        return set_error(LOLA_E_DEVICE, "timing event");
    }
    ctx->timed.push_back(TimedLaunch{kid, units, bytes, ops, a, b});
    return LOLA_OK;
}

// Waits for every recorded launch and adds it to the per-kernel totals.
static int resolve_timing(lola_ctx *ctx) {
    int rc = LOLA_OK;
    for (const TimedLaunch &t : ctx->timed) {
        float ms = 0;
        if (!rc && (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess))
            rc = set_error(LOLA_E_DEVICE, "timing event");
        KernelTotal &k = ctx->ktot[t.kid];
        k.ms += ms;
        k.launches += 1;
        k.units += t.units;
        k.bytes += t.bytes;
        k.ops += t.ops;
        ctx->timing_pool.push_back(t.a);
        ctx->timing_pool.push_back(t.b);
    }
    ctx->timed.clear();
    return rc;
}

static void reset_timing(lola_ctx *ctx) {
    for (KernelTotal &k : ctx->ktot) k = KernelTotal{};
    ctx->timed_jobs = 0;
}

static const char *const KERNEL_NAMES[KID_COUNT] = {
    "ntt_jobs_kernel",      "ks_digits_kernel",       "ks_inner_kernel",  "ks_moddown_kernel",
    "ks_term_kernel",       "ks_fold_kernel",         "ks_term_direct_kernel", "ks_fold_moddown_kernel",
    "ks_modup_kernel",      "ks_hoisted_inner_kernel", "tensor_extend_kernel", "tensor_product_kernel",
    "tensor_round_kernel",  "lin_kernel",             "plain_kernel",     "chain_persistent_kernel",
    "ks_digits_kernel/hoist", "ks_moddown_kernel/hoist"};

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
    int rc = resolve_timing(ctx);
    // the key-switch inner-product stage in whichever form each launch took
    double tot = 0;
    uint64_t nl = 0;
    for (uint32_t k : {KID_KS_INNER, KID_KS_TERM, KID_KS_FOLD, KID_KS_TERM_DIRECT}) {
        tot += ctx->ktot[k].ms;
        nl += k == KID_KS_FOLD ? 0 : ctx->ktot[k].launches;   // a term launch and its fold are one stage
    }
    *total_ms = tot;
    *launches = nl;
    *jobs = ctx->timed_jobs;
    reset_timing(ctx);
    return rc;
}

int lola_kernel_stats(lola_ctx *ctx, lola_kernel_stat *out, uint32_t cap, uint32_t *n_out) {
    if (!ctx || !n_out || (cap && !out)) return set_error(LOLA_E_INVAL, "null argument");
    int rc = resolve_timing(ctx);
    uint32_t n = 0;
    for (uint32_t k = 0; k < KID_COUNT; ++k) {
        const KernelTotal &t = ctx->ktot[k];
        if (t.launches == 0) continue;
        if (n < cap) out[n] = lola_kernel_stat{KERNEL_NAMES[k], t.ms, t.launches, t.units, t.bytes, t.ops};
        ++n;
    }
    *n_out = n;
    reset_timing(ctx);
    return rc ? rc : (n > cap ? set_error(LOLA_E_INVAL, "more kernels than cap (n_out holds the count)") : LOLA_OK);
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
