// Key switching (relinearisation and Galois rotations), batched over jobs.
//
// For a polynomial x (NTT form, [L][N]) and a key for s' -> s, with digits
// D_i = x mod q_i in [0, q_i):
//   u_m = sum_i D_i * key_i   modulo every q_j and P      (key inner product)
//   out_j = (u_j - [u_P]_P) * P^-1 mod q_j                 (mod-down by P)
// A rotation by the Galois element g applies the automorphism first, which in
// the NTT domain is a fixed permutation of evaluation points, so it is folded
// into the loads of x and of the c0 term.
//
// Three launches per batch, one workgroup per limb-sized unit of work:
//   ks_digits   (L per job):    gather sigma_g(x_i) (kept), INTT -> D_i (coefficients)
//   ks_inner    (L+1 per job):  for target modulus m_j: for each digit i,
//                               reduce D_i mod m_j, NTT (i == j reuses x_i),
//                               multiply-accumulate with the key; for P the
//                               two sums are also brought back to coefficients
//   ks_moddown  (2L per job):   lift [u_P]_P into q_j, NTT, subtract, times
//                               P^-1, add the c0 (or d0 / d1) term and an
//                               optional whole-ciphertext addend (fused
//                               rotate-and-add).
#include "ntt_core.hpp"
#include "program.hpp"

namespace lola {

__device__ __forceinline__ uint32_t perm_src(uint32_t idx, uint32_t g, uint32_t logN) {
    return g > 1 ? galois_src_index(idx, g, logN) : idx;
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_digits_kernel(const KsJob *__restrict__ jobs, uint32_t L,
                                                                      const ModConst *__restrict__ mcs,
                                                                      const TwPair *__restrict__ itw) {
    __shared__ uint32_t sh[1 << LOGN];
    const KsJob job = jobs[blockIdx.y];
    const uint32_t i = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const ModConst mc = mcs[i];
    const GBuf xi = gbuf(job.x + ((size_t)i << LOGN), 1u << LOGN);
    const GBuf Xp = gbuf(job.scratch + ((size_t)(L + i) << LOGN), 1u << LOGN);
    uint32_t x[NTT_E];
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = gld(xi, perm_src(spectral_index<LOGN>(tid, r), job.galois, LOGN));
    store_spectral<LOGN>(Xp, tid, x);  // sigma_g(x_i) in NTT form: the digit's own-modulus transform
    ntt_inv_regs<LOGN>(x, tid, sh, itw + ((size_t)i << LOGN), mc);
    const GBuf D = gbuf(job.scratch + ((size_t)i << LOGN), 1u << LOGN);
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) gst(D, natural_index<LOGN>(tid, r), x[r]);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_inner_kernel(const KsJob *__restrict__ jobs, uint32_t L,
                                                                     const ModConst *__restrict__ mcs,
                                                                     const TwPair *__restrict__ tw,
                                                                     const TwPair *__restrict__ itw) {
    constexpr uint32_t N = 1u << LOGN;
    __shared__ uint32_t sh[N];
    const KsJob job = jobs[blockIdx.y];
    const uint32_t j = blockIdx.x;  // target modulus: q_j (j < L) or P (j == L)
    const ModConst mc = mcs[j];
    const uint32_t M = L + 1;
    // 64-bit accumulators: every term is x * key with x < q (the transform's
    // output is canonical) and key < q, so at most 12 digits sum below
    // 12 q^2 < 2^64; one Montgomery reduction at the end (keys are stored
    // times 2^32).
    uint64_t a0[NTT_E], a1[NTT_E];
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) a0[r] = a1[r] = 0;
    for (uint32_t i = 0; i < L; ++i) {
        // Every index below depends only on the thread id; an opaque copy per
        // iteration keeps the compiler from hoisting all of them (and the
        // transform's LDS addresses) out of the loop, which would not fit in
        // the 128 registers a 1024-thread workgroup allows.
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        uint32_t x[NTT_E];
        if (i == j) {
            load_spectral<LOGN>(gbuf(job.scratch + ((size_t)(L + i) << LOGN), N), tid, x);
        } else {
            const GBuf D = gbuf(job.scratch + ((size_t)i << LOGN), N);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) x[r] = reduce32(gld(D, natural_index<LOGN>(tid, r)), mc.q, mc.one_shoup);
            // The twiddle table does not change with i; an opaque copy of j
            // keeps the compiler from hoisting every twiddle load of the
            // transform out of the loop.
            uint32_t jj = j;
            asm volatile("" : "+s"(jj));
            ntt_fwd_regs<LOGN>(x, tid, sh, tw + ((size_t)jj << LOGN), mc.q);
        }
        // Key offsets pass through an opaque copy placed after the transform,
        // so the 32 key loads are not scheduled ahead of it.
        uint32_t koff = i * 2 * M + j;
        asm volatile("" : "+s"(koff));
        const GBuf kb = gbuf(job.key + ((size_t)koff << LOGN), N);
        const GBuf ka = gbuf(job.key + ((size_t)(koff + M) << LOGN), N);
        uint32_t kbv[NTT_E], kav[NTT_E];
        load_spectral<LOGN>(kb, tid, kbv);
        load_spectral<LOGN>(ka, tid, kav);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) {
            a0[r] += (uint64_t)x[r] * kbv[r];
            a1[r] += (uint64_t)x[r] * kav[r];
        }
    }
    const uint32_t tid = threadIdx.x;
    uint32_t u[NTT_E];
    if (j < L) {
        const GBuf U0 = gbuf(job.scratch + ((size_t)(2 * L + j) << LOGN), N);
        const GBuf U1 = gbuf(job.scratch + ((size_t)(3 * L + j) << LOGN), N);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a0[r], (uint32_t)(a0[r] >> 32)}, mc);
        store_spectral<LOGN>(U0, tid, u);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a1[r], (uint32_t)(a1[r] >> 32)}, mc);
        store_spectral<LOGN>(U1, tid, u);
    } else {
        const GBuf UP = gbuf(job.scratch + ((size_t)(4 * L) << LOGN), N);
        const GBuf UP1 = gbuf(job.scratch + ((size_t)(4 * L + 1) << LOGN), N);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a0[r], (uint32_t)(a0[r] >> 32)}, mc);
        ntt_inv_regs<LOGN>(u, tid, sh, itw + ((size_t)j << LOGN), mc);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(UP, natural_index<LOGN>(tid, r), u[r]);
        uint32_t tid2 = tid;
        asm volatile("" : "+v"(tid2));
        uint32_t jj = j;
        asm volatile("" : "+s"(jj));
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a1[r], (uint32_t)(a1[r] >> 32)}, mc);
        ntt_inv_regs<LOGN>(u, tid2, sh, itw + ((size_t)jj << LOGN), mc);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(UP1, natural_index<LOGN>(tid2, r), u[r]);
    }
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_moddown_kernel(const KsJob *__restrict__ jobs, uint32_t L,
                                                                       const ModConst *__restrict__ mcs,
                                                                       const TwPair *__restrict__ tw,
                                                                       const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[1 << LOGN];
    const KsJob job = jobs[blockIdx.z];
    const uint32_t j = blockIdx.x, c = blockIdx.y;
    const uint32_t tid = threadIdx.x;
    const ModConst mc = mcs[j];
    const uint32_t P = mcs[L].q, halfP = P >> 1;
    const uint32_t Pq = mrc->Pq[j];
    constexpr uint32_t N = 1u << LOGN;
    const GBuf UP = gbuf(job.scratch + ((size_t)(4 * L + c) << LOGN), N);
    uint32_t x[NTT_E];
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) {
        const uint32_t v = gld(UP, natural_index<LOGN>(tid, r));
        const uint32_t vr = reduce32(v, mc.q, mc.one_shoup);
        x[r] = v > halfP ? sub_mod(vr, Pq, mc.q) : vr;  // [u_P]_P mod q_j
    }
    ntt_fwd_regs<LOGN>(x, tid, sh, tw + ((size_t)j << LOGN), mc.q);
    const GBuf U = gbuf(job.scratch + ((size_t)((2 + c) * L + j) << LOGN), N);
    const uint32_t *add = c == 0 ? job.add0 : job.add1;
    const uint32_t g = c == 0 ? job.galois : 0u;
    const uint32_t pinv = mrc->Pinvq[j], pinvp = mrc->Pinvqp[j];
    const GBuf out = gbuf(job.out + ((size_t)(c * L + j) << LOGN), N);
    const bool has_add = add != nullptr, has_addc = job.addct != nullptr;
    const GBuf addj = gbuf(has_add ? add + ((size_t)j << LOGN) : job.out, has_add ? N : 0u);
    const GBuf addc = gbuf(has_addc ? job.addct + ((size_t)(c * L + j) << LOGN) : job.out, has_addc ? N : 0u);
    uint32_t uu[NTT_E];
    load_spectral<LOGN>(U, tid, uu);
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = shoup(sub_mod(uu[r], x[r], mc.q), pinv, pinvp, mc.q);
    if (has_add) {
#pragma unroll
        for (int r = 0; r < NTT_E; ++r)
            x[r] = add_mod(x[r], gld(addj, perm_src(spectral_index<LOGN>(tid, r), g, LOGN)), mc.q);
    }
    if (has_addc) {
        load_spectral<LOGN>(addc, tid, uu);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = add_mod(x[r], uu[r], mc.q);
    }
    store_spectral<LOGN>(out, tid, x);
}

size_t ks_scratch_words(const lola_ctx *ctx) { return (size_t)(4 * ctx->L + 2) * ctx->N; }

int launch_keyswitch(lola_ctx *ctx, const KsJob *d_jobs, uint32_t n, hipStream_t s) {
    const uint32_t L = ctx->L;
    const dim3 block(ctx->N / NTT_E);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (ctx->timing) {
        int rc = timing_pair(ctx, &t0, &t1);
        if (rc) return rc;
        ctx->timed_jobs += n;
    }
#define LOLA_KS_CASE(LG)                                                                                     \
    case LG:                                                                                                 \
        hipLaunchKernelGGL(ks_digits_kernel<LG>, dim3(L, n), block, 0, s, d_jobs, L, ctx->d_mc, ctx->d_itw);  \
        if (t0) LOLA_HIP(hipEventRecord(t0, s));                                                             \
        hipLaunchKernelGGL(ks_inner_kernel<LG>, dim3(L + 1, n), block, 0, s, d_jobs, L, ctx->d_mc, ctx->d_tw,  \
                           ctx->d_itw);                                                                       \
        if (t1) LOLA_HIP(hipEventRecord(t1, s));                                                             \
        hipLaunchKernelGGL(ks_moddown_kernel<LG>, dim3(L, 2, n), block, 0, s, d_jobs, L, ctx->d_mc, ctx->d_tw, \
                           ctx->d_mrc);                                                                       \
        break;
    switch (ctx->logN) {
        LOLA_KS_CASE(10)
        LOLA_KS_CASE(11)
        LOLA_KS_CASE(12)
        LOLA_KS_CASE(13)
        LOLA_KS_CASE(14)
        default: return set_error(LOLA_E_PARAMS, "unsupported N");
    }
#undef LOLA_KS_CASE
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

// Jobs per launch: bounds the scratch arena ((4L+2) N words per job).
static constexpr uint32_t KS_CHUNK = 128;

void program_keyswitch(const lola_ctx *ctx, Program &p, std::vector<KsJob> jobs, uint32_t *scratch,
                       uint32_t chunk) {
    const size_t per = ks_scratch_words(ctx);
    for (size_t off = 0; off < jobs.size(); off += chunk) {
        const size_t n = std::min<size_t>(chunk, jobs.size() - off);
        std::vector<KsJob> part(jobs.begin() + off, jobs.begin() + off + n);
        for (size_t k = 0; k < n; ++k) part[k].scratch = scratch + per * k;
        p.launch(LK_KS, part);
        p.ks_jobs += n;
    }
}

int keyswitch_host_jobs(lola_ctx *ctx, std::vector<KsJob> &jobs, hipStream_t s) {
    const size_t per = ks_scratch_words(ctx);
    for (size_t off = 0; off < jobs.size(); off += KS_CHUNK) {
        const uint32_t n = (uint32_t)std::min<size_t>(KS_CHUNK, jobs.size() - off);
        void *buf = nullptr;
        int rc = scratch_get(ctx, per * n * 4, &buf);
        if (rc) return rc;
        Program p;
        program_keyswitch(ctx, p, std::vector<KsJob>(jobs.begin() + off, jobs.begin() + off + n),
                          (uint32_t *)buf, n);
        if ((rc = program_run_now(ctx, p, s))) return rc;
    }
    return LOLA_OK;
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_reserve(lola_ctx *ctx, uint32_t n_ct) {
    if (!ctx) return set_error(LOLA_E_INVAL, "null argument");
    void *buf = nullptr;
    const size_t per = std::max<size_t>(ks_scratch_words(ctx), mul_scratch_words(ctx));
    return scratch_get(ctx, per * std::min<uint32_t>(std::max<uint32_t>(n_ct, 1), KS_CHUNK) * 4, &buf);
}

int lola_keyswitch_batch(lola_ctx *ctx, const lola_ks_desc *d, uint32_t n, lola_stream stream) {
    if (!ctx || (!d && n)) return set_error(LOLA_E_INVAL, "null argument");
    const size_t P = (size_t)ctx->L * ctx->N;
    std::vector<KsJob> jobs(n);
    for (uint32_t k = 0; k < n; ++k) {
        if (!d[k].in_dev || !d[k].key_dev || !d[k].out_dev) return set_error(LOLA_E_NOKEY, "null key or buffer in batch");
        if (d[k].galois != 0 && (!(d[k].galois & 1) || d[k].galois >= 2 * ctx->N))
            return set_error(LOLA_E_INVAL, "bad Galois element");
        if (d[k].galois == 0)
            jobs[k] = KsJob{d[k].in_dev + 2 * P, d[k].key_dev, d[k].in_dev, d[k].in_dev + P, nullptr, d[k].out_dev, nullptr, 0, 0};
        else
            jobs[k] = KsJob{d[k].in_dev + P, d[k].key_dev, d[k].in_dev, nullptr, nullptr, d[k].out_dev, nullptr, d[k].galois, 0};
    }
    return keyswitch_host_jobs(ctx, jobs, (hipStream_t)stream);
}

int lola_relin(lola_ctx *ctx, const uint32_t *rlk, const uint32_t *in3, uint32_t *out, lola_stream stream) {
    if (!rlk) return set_error(LOLA_E_NOKEY, "missing relinearisation key");
    lola_ks_desc d{in3, rlk, out, 0, 0};
    return lola_keyswitch_batch(ctx, &d, 1, stream);
}

int lola_rotate(lola_ctx *ctx, const uint32_t *gk, uint32_t galois, const uint32_t *ct, uint32_t *out,
                lola_stream stream) {
    if (!gk) return set_error(LOLA_E_NOKEY, "missing Galois key");
    if (galois == 0) return set_error(LOLA_E_INVAL, "Galois element 0");
    lola_ks_desc d{ct, gk, out, galois, 0};
    return lola_keyswitch_batch(ctx, &d, 1, stream);
}

}  // extern "C"
