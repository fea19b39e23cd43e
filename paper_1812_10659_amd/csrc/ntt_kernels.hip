// Batched limb NTTs: each workgroup transforms LPW (limb, prime) jobs in turn.
//
// Variants: the radix split (how the log2(N) stages group into register
// passes, see NttShape) and the tile (jobs per workgroup) are template
// choices; every combination in the list below is compiled, and the context
// selects one (lola_ntt_set_variant, or lola_ntt_autotune, which times them
// all on the device and keeps the fastest).  All variants read and write the
// same global layouts, so their results are identical word for word.
#include <algorithm>
#include <cstring>

#include "lola_internal.hpp"
#include "ntt_core.hpp"

namespace lola {

// Jobs without descriptors: job k transforms limb k of the contiguous array
// `in` into limb k of `out`, under prime k mod `cycle` (the limbs of
// consecutive [..][L][N] polynomials), all with the same flags.
struct NttStrided {
    const uint32_t *in;
    uint32_t *out;
    uint32_t cycle, flags;
};

// Launch bound: at least 8 waves per SIMD, i.e. at most 64 VGPRs, so two
// 1024-thread workgroups (64 KiB of LDS each) fit one CU at N = 16384.
// jobs: device descriptors, or null for the strided jobs of `sd`.
template <int LOGN, int SPLIT, int LPW>
__global__ __launch_bounds__((1 << LOGN) / NTT_E, 8) void ntt_jobs_kernel(
    const NttJob *__restrict__ jobs, uint32_t n, const ModConst *__restrict__ mcs, const TwPair *__restrict__ tw,
    const TwPair *__restrict__ itw, uint32_t t, const MrcConst *__restrict__ mrc, NttStrided sd) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, false>()];   // plain placement
    constexpr uint32_t N = 1u << LOGN;
    for (uint32_t k = 0; k < (uint32_t)LPW; ++k) {
        // the same for every thread of the workgroup: the exit is uniform;
        // each transform starts with a workgroup barrier before its first
        // LDS write, so consecutive jobs can share sh
        const uint32_t jb = blockIdx.x * LPW + k;
        if (jb >= n) return;
        const NttJob job = jobs ? jobs[jb]
                                : NttJob{sd.in + ((size_t)jb << LOGN), sd.out + ((size_t)jb << LOGN), jb % sd.cycle,
                                         sd.flags};
        const ModConst mc = mcs[job.prime];
        const uint32_t tid = threadIdx.x;
        const size_t toff = (size_t)job.prime << LOGN;
        const GBuf src = gbuf(job.src, N), dst = gbuf(job.dst, N);
        uint32_t x[NTT_E];
        if (!(job.flags & NTT_INVERSE)) {
            // All 16 loads first, then the (workgroup-uniform) source
            // conversions as passes of their own: a flag test between the
            // loads splits them into separate blocks, each waiting for its
            // load, which measured 1.4x slower for the whole kernel.
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) x[r] = gld(src, natural_index<LOGN, SPLIT>(tid, r));
            if (job.flags & NTT_SRC_SIGNED_T) {
                // [v]_t mod q: values above t/2 stand for v - t
#pragma unroll
                for (int r = 0; r < NTT_E; ++r) x[r] = (x[r] > (t >> 1)) ? mc.q - (t - x[r]) : x[r];
            }
            if (job.flags & NTT_SRC_SIGNED32) {
#pragma unroll
                for (int r = 0; r < NTT_E; ++r) {
                    const int32_t sv = (int32_t)x[r];
                    x[r] = sv < 0 ? mc.q - (uint32_t)(-sv) : (uint32_t)sv;
                }
            }
            if (job.flags & NTT_SRC_REDUCE) {
#pragma unroll
                for (int r = 0; r < NTT_E; ++r) x[r] = reduce32(x[r], mc.q, mc.one_shoup);
            }
            ntt_fwd_regs<LOGN, false, SPLIT>(x, tid, sh, tw + toff, mc.q);
            if (job.flags & NTT_MUL_DELTA) {
                const uint32_t d = mrc->deltaq[job.prime], dp = mrc->deltaqp[job.prime];
#pragma unroll
                for (int r = 0; r < NTT_E; ++r) x[r] = shoup(x[r], d, dp, mc.q);
            }
            if (job.flags & NTT_TO_MONT) {
#pragma unroll
                for (int r = 0; r < NTT_E; ++r) x[r] = shoup(x[r], mc.r_mod, mc.r_shoup, mc.q);
            }
            store_spectral<LOGN, SPLIT>(dst, tid, x);
        } else {
            load_spectral<LOGN, SPLIT>(src, tid, x);
            if (job.flags & NTT_FROM_MONT) {
#pragma unroll
                for (int r = 0; r < NTT_E; ++r) x[r] = mont_mul(x[r], 1u, mc.q, mc.qneg_inv);
            }
            ntt_inv_regs<LOGN, SPLIT>(x, tid, sh, itw + toff, mc);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) gst(dst, natural_index<LOGN, SPLIT>(tid, r), x[r]);
        }
    }
}

// The split written out as digits (SPLIT = 0 names the default split).
constexpr uint32_t split_code(int logn, int split) {
    uint32_t c = 0;
    for (int p = 0; p < split_npass(logn, split); ++p) c = c * 10 + (uint32_t)split_width(logn, split, p);
    return c;
}

using NttKernelFn = void (*)(const NttJob *, uint32_t, const ModConst *, const TwPair *, const TwPair *, uint32_t,
                             const MrcConst *, NttStrided);
struct NttVariant {
    uint32_t split, lpw;
    NttKernelFn fn;
};

#define LOLA_NTT_V(LG, SP)                                           \
    NttVariant{split_code(LG, SP), 1, ntt_jobs_kernel<LG, SP, 1>},   \
        NttVariant{split_code(LG, SP), 2, ntt_jobs_kernel<LG, SP, 2>}, \
        NttVariant{split_code(LG, SP), 4, ntt_jobs_kernel<LG, SP, 4>}
// Candidates per N: the default first (index 0), then other orders of the
// same pass widths and splits with 3-stage passes.
static const NttVariant NTT_V10[] = {LOLA_NTT_V(10, 0), LOLA_NTT_V(10, 244), LOLA_NTT_V(10, 424),
                                     LOLA_NTT_V(10, 433), LOLA_NTT_V(10, 334)};
static const NttVariant NTT_V11[] = {LOLA_NTT_V(11, 0), LOLA_NTT_V(11, 344), LOLA_NTT_V(11, 434),
                                     LOLA_NTT_V(11, 3332)};
static const NttVariant NTT_V12[] = {LOLA_NTT_V(12, 0), LOLA_NTT_V(12, 3333), LOLA_NTT_V(12, 4332),
                                     LOLA_NTT_V(12, 2334)};
static const NttVariant NTT_V13[] = {LOLA_NTT_V(13, 0), LOLA_NTT_V(13, 4414), LOLA_NTT_V(13, 1444),
                                     LOLA_NTT_V(13, 4432), LOLA_NTT_V(13, 4333), LOLA_NTT_V(13, 3334)};
static const NttVariant NTT_V14[] = {LOLA_NTT_V(14, 0),    LOLA_NTT_V(14, 4424), LOLA_NTT_V(14, 4244),
                                     LOLA_NTT_V(14, 2444), LOLA_NTT_V(14, 4433), LOLA_NTT_V(14, 3443),
                                     LOLA_NTT_V(14, 3344)};
#undef LOLA_NTT_V

static bool ntt_variant_list(uint32_t logN, const NttVariant **v, uint32_t *count) {
#define LOLA_NTT_LIST(LG)                                      \
    case LG:                                                   \
        *v = NTT_V##LG;                                        \
        *count = (uint32_t)(sizeof(NTT_V##LG) / sizeof(NTT_V##LG[0])); \
        return true;
    switch (logN) {
        LOLA_NTT_LIST(10)
        LOLA_NTT_LIST(11)
        LOLA_NTT_LIST(12)
        LOLA_NTT_LIST(13)
        LOLA_NTT_LIST(14)
        default: return false;
    }
#undef LOLA_NTT_LIST
}

static int launch_ntt_any(lola_ctx *ctx, const NttJob *d_jobs, NttStrided sd, int n, hipStream_t s) {
    if (n <= 0) return LOLA_OK;
    const NttVariant *vs = nullptr;
    uint32_t count = 0;
    if (!ntt_variant_list(ctx->logN, &vs, &count)) return set_error(LOLA_E_PARAMS, "unsupported N");
    const NttVariant &v = vs[ctx->ntt_variant < count ? ctx->ntt_variant : 0];
    uint32_t nj = (uint32_t)n;
    const ModConst *mc = ctx->d_mc;
    const TwPair *tw = ctx->d_tw, *itw = ctx->d_itw;
    uint32_t t = ctx->t;
    const MrcConst *mrc = ctx->d_mrc;
    void *args[] = {(void *)&d_jobs, (void *)&nj, (void *)&mc, (void *)&tw, (void *)&itw, (void *)&t, (void *)&mrc,
                    (void *)&sd};
    LOLA_TIMED(ctx, s, KID_NTT, nj, 8.0 * ctx->N * nj, xform_ops(ctx) * nj,
               LOLA_HIP(hipLaunchKernel((const void *)v.fn, dim3((nj + v.lpw - 1) / v.lpw), dim3(ctx->N / NTT_E),
                                        args, 0, s)));
    return LOLA_OK;
}

int launch_ntt_jobs_dev(lola_ctx *ctx, const NttJob *d_jobs, int n, hipStream_t s) {
    return launch_ntt_any(ctx, d_jobs, NttStrided{}, n, s);
}

// n limbs of `in` to n limbs of `out`, limb k under prime k mod cycle: no
// descriptors to upload.
int launch_ntt_strided(lola_ctx *ctx, const uint32_t *in, uint32_t *out, uint32_t n, uint32_t cycle,
                       uint32_t flags, hipStream_t s) {
    if (cycle == 0 || cycle > ctx->nprimes()) return set_error(LOLA_E_INVAL, "prime cycle out of range");
    return launch_ntt_any(ctx, nullptr, NttStrided{in, out, cycle, flags}, (int)n, s);
}

// Residues for tuning: limb k holds pseudo-random values below its prime.
__global__ void ntt_tune_fill_kernel(uint32_t *x, uint32_t n_limbs, uint32_t logN, uint32_t L,
                                     const ModConst *__restrict__ mcs) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ((size_t)n_limbs << logN)) return;
    uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
    const uint32_t limb = (uint32_t)(i >> logN);
    x[i] = (uint32_t)(h % mcs[limb % L].q);
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

int lola_ntt_variants(const lola_ctx *ctx, lola_ntt_variant *out, uint32_t cap, uint32_t *count) {
    if (!ctx || !count || (cap && !out)) return set_error(LOLA_E_INVAL, "null argument");
    const NttVariant *vs = nullptr;
    uint32_t nv = 0;
    if (!ntt_variant_list(ctx->logN, &vs, &nv)) return set_error(LOLA_E_PARAMS, "unsupported N");
    *count = nv;
    for (uint32_t k = 0; k < nv && k < cap; ++k) out[k] = lola_ntt_variant{vs[k].split, vs[k].lpw, 0.0f};
    return LOLA_OK;
}

int lola_ntt_get_variant(const lola_ctx *ctx, uint32_t *index) {
    if (!ctx || !index) return set_error(LOLA_E_INVAL, "null argument");
    *index = ctx->ntt_variant;
    return LOLA_OK;
}

int lola_ntt_set_variant(lola_ctx *ctx, uint32_t index) {
    if (!ctx) return set_error(LOLA_E_INVAL, "null argument");
    const NttVariant *vs = nullptr;
    uint32_t nv = 0;
    if (!ntt_variant_list(ctx->logN, &vs, &nv)) return set_error(LOLA_E_PARAMS, "unsupported N");
    if (index >= nv) return set_error(LOLA_E_INVAL, "NTT variant index out of range");
    ctx->ntt_variant = index;
    return LOLA_OK;
}

int lola_ntt_autotune(lola_ctx *ctx, uint32_t n_limbs, uint32_t reps, lola_ntt_variant *out, uint32_t cap,
                      uint32_t *chosen, lola_stream stream) {
    if (!ctx || !chosen || (cap && !out)) return set_error(LOLA_E_INVAL, "null argument");
    if (n_limbs == 0 || n_limbs > 65536 || reps == 0 || reps > 1000)
        return set_error(LOLA_E_INVAL, "n_limbs in [1, 65536], reps in [1, 1000]");
    const NttVariant *vs = nullptr;
    uint32_t nv = 0;
    if (!ntt_variant_list(ctx->logN, &vs, &nv)) return set_error(LOLA_E_PARAMS, "unsupported N");
    hipStream_t s = (hipStream_t)stream;
    const size_t words = (size_t)n_limbs * ctx->N;
    uint32_t *buf = nullptr;   // in, spectral, back, reference spectral
    NttJob *d_jobs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const uint32_t saved = ctx->ntt_variant;
    std::vector<uint32_t> h_in(words), h_a(words), h_b(words);
    std::vector<float> ms(nv, 0.0f);
    int rc = LOLA_OK;
    auto fail = [&](int code) {
        if (buf) (void)hipFree(buf);
        if (d_jobs) (void)hipFree(d_jobs);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        ctx->ntt_variant = saved;
        return code;
    };
    if (hipMalloc(&buf, 4 * words * 4) != hipSuccess) return fail(set_error(LOLA_E_NOMEM, "autotune buffers"));
    if (hipMalloc(&d_jobs, 2 * (size_t)n_limbs * sizeof(NttJob)) != hipSuccess)
        return fail(set_error(LOLA_E_NOMEM, "autotune descriptors"));
    uint32_t *in = buf, *spec = buf + words, *back = buf + 2 * words, *ref = buf + 3 * words;
    std::vector<NttJob> jobs(2 * (size_t)n_limbs);
    for (uint32_t k = 0; k < n_limbs; ++k) {
        const uint32_t pr = k % ctx->L;
        jobs[k] = NttJob{in + (size_t)k * ctx->N, spec + (size_t)k * ctx->N, pr, 0u};
        jobs[n_limbs + k] = NttJob{spec + (size_t)k * ctx->N, back + (size_t)k * ctx->N, pr, NTT_INVERSE};
    }
    if (hipMemcpy(d_jobs, jobs.data(), jobs.size() * sizeof(NttJob), hipMemcpyHostToDevice) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(set_error(LOLA_E_DEVICE, "autotune setup"));
    hipLaunchKernelGGL(ntt_tune_fill_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, in, n_limbs,
                       ctx->logN, ctx->L, ctx->d_mc);
    auto run = [&](uint32_t v) -> int {
        ctx->ntt_variant = v;
        int r = launch_ntt_jobs_dev(ctx, d_jobs, (int)n_limbs, s);
        if (!r) r = launch_ntt_jobs_dev(ctx, d_jobs + n_limbs, (int)n_limbs, s);
        return r;
    };
    // reference: the default variant; its inverse must give the input back
    if ((rc = run(0))) return fail(rc);
    if (hipMemcpyAsync(ref, spec, words * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h_in.data(), in, words * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_a.data(), ref, words * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_b.data(), back, words * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(set_error(LOLA_E_DEVICE, "autotune reference"));
    if (memcmp(h_in.data(), h_b.data(), words * 4) != 0)
        return fail(set_error(LOLA_E_DEVICE, "autotune: default NTT variant does not invert"));
    std::vector<uint32_t> h_s(words);
    for (uint32_t v = 0; v < nv; ++v) {
        // every variant must reproduce the reference words before it is timed
        if ((rc = run(v))) return fail(rc);
        if (hipMemcpyAsync(h_s.data(), spec, words * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(h_b.data(), back, words * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(set_error(LOLA_E_DEVICE, "autotune readback"));
        if (memcmp(h_s.data(), h_a.data(), words * 4) != 0 || memcmp(h_b.data(), h_in.data(), words * 4) != 0)
            return fail(set_error(LOLA_E_DEVICE, "autotune: NTT variant " + std::to_string(vs[v].split) + "/" +
                                                     std::to_string(vs[v].lpw) + " differs from the default"));
        if (hipEventRecord(e0, s) != hipSuccess) return fail(set_error(LOLA_E_DEVICE, "autotune event"));
        for (uint32_t r = 0; r < reps; ++r)
            if ((rc = run(v))) return fail(rc);
        float t = 0;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            return fail(set_error(LOLA_E_DEVICE, "autotune timing"));
        ms[v] = t / (float)reps;
    }
    uint32_t best = 0;
    for (uint32_t v = 1; v < nv; ++v)
        if (ms[v] < ms[best]) best = v;
    for (uint32_t k = 0; k < nv && k < cap; ++k) out[k] = lola_ntt_variant{vs[k].split, vs[k].lpw, ms[k]};
    fail(LOLA_OK);   // frees the buffers and restores the variant
    ctx->ntt_variant = best;
    *chosen = best;
    return LOLA_OK;
}

int lola_ntt_limbs(lola_ctx *ctx, const uint32_t *in_dev, uint32_t *out_dev, uint32_t n_limbs,
                   const uint32_t *prime_idx_host, int inverse, lola_stream stream) {
    if (!ctx || !in_dev || !out_dev || !prime_idx_host) return set_error(LOLA_E_INVAL, "null argument");
    // limb k under prime k mod L (consecutive polynomials of L limbs): no
    // descriptors at all
    bool cyclic = true;
    for (uint32_t k = 0; k < n_limbs && cyclic; ++k) cyclic = prime_idx_host[k] == k % ctx->L;
    if (cyclic) return launch_ntt_strided(ctx, in_dev, out_dev, n_limbs, ctx->L, inverse ? NTT_INVERSE : 0u,
                                          (hipStream_t)stream);
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
    return launch_ntt_strided(ctx, in_dev, out_dev, n_polys * ctx->L, ctx->L, NTT_INVERSE, (hipStream_t)stream);
}

int lola_from_coeff(lola_ctx *ctx, const uint32_t *in_dev, uint32_t n_polys, uint32_t *out_dev,
                    lola_stream stream) {
    if (!ctx || !in_dev || !out_dev) return set_error(LOLA_E_INVAL, "null argument");
    return launch_ntt_strided(ctx, in_dev, out_dev, n_polys * ctx->L, ctx->L, NTT_SRC_REDUCE, (hipStream_t)stream);
}

}  // extern "C"
