// Batched element-wise jobs, the program runner, and kernel timing.
#include "program.hpp"

namespace lola {

// dst[d] = sum_k w[d]_k src_k (+ add[d] on component 0) for the job's n_dst
// outputs.  grid (2LN/4/256, jobs)
//
// A block's 1024 words lie in one limb (N >= 1024), so the limb and the
// weights are uniform and come from scalar loads.  Sources are taken in
// groups of LIN_GROUP with all their loads issued before any product: a
// group past the last source repeats the last source's address with weight
// 0 (a zero term), which keeps the group one straight block instead of a
// test and a wait per source.  Each source word is loaded once for all the
// job's outputs.  The weights are in Montgomery form (w' = w 2^32 mod q),
// every term x w' (< q^2 < 2^60) is added into a 64-bit accumulator with one
// multiply-add, and one Montgomery reduction at the end gives
// sum_k x_k w_k mod q.  Every LIN_LAZY terms the accumulator is brought back
// below q^2 without changing its residue: r = acc 2^-32 mod q, acc = r (2^32
// mod q), so at most LIN_LAZY terms and one such value (13 q^2 < 2^64) are
// ever summed.
constexpr uint32_t LIN_GROUP = 4, LIN_LAZY = 12;
static_assert(LIN_LAZY % LIN_GROUP == 0, "reductions fall between groups of sources");

__global__ void lin_kernel(const LinJob *__restrict__ jobs, uint32_t logN, uint32_t L,
                           const ModConst *__restrict__ mcs) {
    const LinJob &job = jobs[blockIdx.y];
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n4 = ((size_t)2 * L << logN) / 4;
    if (i >= n4) return;
    const uint32_t cl = (uint32_t)(((size_t)blockIdx.x * blockDim.x * 4) >> logN);   // component * L + limb
    const uint32_t limb = cl % L;
    const ModConst mc = mcs[limb];
    const uint32_t q = mc.q;
    const uint32_t n = job.n_src, nd = job.n_dst;
    uint64_t acc[LIN_OUT][4];
#pragma unroll
    for (uint32_t d = 0; d < LIN_OUT; ++d)
        for (uint32_t c = 0; c < 4; ++c) acc[d][c] = 0;
    for (uint32_t k0 = 0; k0 < n; k0 += LIN_GROUP) {
        uint4 x[LIN_GROUP];
#pragma unroll
        for (uint32_t b = 0; b < LIN_GROUP; ++b) x[b] = ((const uint4 *)job.srcs[min(k0 + b, n - 1)])[i];
        const bool reduce = (k0 + LIN_GROUP) % LIN_LAZY == 0 && k0 + LIN_GROUP < n;
#pragma unroll
        for (uint32_t d = 0; d < LIN_OUT; ++d) {
            if (d >= nd) break;
            const uint32_t *wt = job.w[d];
#pragma unroll
            for (uint32_t b = 0; b < LIN_GROUP; ++b) {
                // the clamped source's Montgomery weight, masked to 0 past the last one
                const uint32_t k = min(k0 + b, n - 1), mask = 0u - (uint32_t)(k0 + b < n);
                const uint32_t w = wt[(2 * k + 1) * L + limb] & mask;
                acc[d][0] += (uint64_t)x[b].x * w;
                acc[d][1] += (uint64_t)x[b].y * w;
                acc[d][2] += (uint64_t)x[b].z * w;
                acc[d][3] += (uint64_t)x[b].w * w;
            }
            if (reduce) {
#pragma unroll
                for (uint32_t c = 0; c < 4; ++c)
                    acc[d][c] = (uint64_t)acc_reduce_mont(Acc64{(uint32_t)acc[d][c], (uint32_t)(acc[d][c] >> 32)}, mc) *
                                mc.r_mod;
            }
        }
    }
#pragma unroll
    for (uint32_t d = 0; d < LIN_OUT; ++d) {
        if (d >= nd) break;
        uint32_t r[4];
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c) r[c] = acc_reduce_mont(Acc64{(uint32_t)acc[d][c], (uint32_t)(acc[d][c] >> 32)}, mc);
        if (job.add[d] && cl < L) {
            const uint4 y = ((const uint4 *)job.add[d])[i];
            r[0] = add_mod(r[0], y.x, q), r[1] = add_mod(r[1], y.y, q), r[2] = add_mod(r[2], y.z, q),
            r[3] = add_mod(r[3], y.w, q);
        }
        ((uint4 *)job.dst[d])[i] = make_uint4(r[0], r[1], r[2], r[3]);
    }
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
// LN words), every output ciphertext is written; each source word takes a
// modular product and an add per output (counted so although the kernel
// multiply-adds into 64 bits and reduces every 16 terms), each constant word
// an add.
int launch_lin_dev(lola_ctx *ctx, const LinJob *d, uint32_t n, const uint64_t *aux, hipStream_t s) {
    const size_t n4 = (size_t)2 * ctx->L * ctx->N / 4;
    const double ln = (double)ctx->L * ctx->N;
    LOLA_TIMED(ctx, s, KID_LIN, aux[4], 4 * ln * (2.0 * (aux[1] + aux[4]) + aux[3]),
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
