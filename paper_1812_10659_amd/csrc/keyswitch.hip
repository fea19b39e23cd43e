// Key switching (relinearisation and Galois rotations), batched over jobs.
//
// Three launches per batch, one workgroup per limb-sized unit of work (the
// stages themselves are in ks_core.hpp):
//   ks_digits   (L per job):    gather sigma_g(x_i) (kept), INTT -> D_i (coefficients)
//   ks_inner    (L+1 per job):  for target modulus m_j: for each digit i,
//                               reduce D_i mod m_j, NTT (i == j reuses x_i),
//                               multiply-accumulate with the key; for P the
//                               two sums are also brought back to coefficients
//   ks_moddown  (2L per job):   lift [u_P]_P into q_j, NTT, subtract, times
//                               P^-1, add the c0 (or d0 / d1) term and an
//                               optional whole-ciphertext addend (fused
//                               rotate-and-add).
#include <algorithm>

#include "ks_core.hpp"
#include "program.hpp"

namespace lola {

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_digits_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                      uint32_t L, const ModConst *__restrict__ mcs,
                                                                      const TwPair *__restrict__ itw) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN>()];
    const JobUnit ju = xcd_job_unit(blockIdx.x, L, n);
    if (ju.job >= n) return;
    const KsJob job = jobs[ju.job];
    const uint32_t i = ju.unit;
    ks_stage_digit<LOGN>(job.x, job.galois, job.scratch, i, L, sh, mcs[i], itw);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_inner_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                     uint32_t L, const ModConst *__restrict__ mcs,
                                                                     const TwPair *__restrict__ tw,
                                                                     const TwPair *__restrict__ itw) {
    __shared__ uint32_t sh[2 << LOGN];   // two halves for the plain placement
    const JobUnit ju = xcd_job_unit(blockIdx.x, L + 1, n);
    if (ju.job >= n) return;
    const KsJob job = jobs[ju.job];
    // target modulus: q_j (j < L) or P (j == L); the special prime's unit,
    // half again as long as the others, is dispatched first of its job so the
    // launch's tail holds short units
    const uint32_t j = ju.unit == 0 ? L : ju.unit - 1;
    ks_stage_inner<LOGN>(job.key, job.scratch, j, L, sh, mcs[j], tw, itw);
}

// Latency form of the inner stage (launches of at most KS_TERM_MAX_JOBS
// jobs): L (L+1) workgroups per job, one digit term each, then 2 (L+1) that
// fold the terms.  The special prime's units come first, as above.  Grid =
// jobs x units, workgroup k taking unit k mod units of job k / units: the
// units of one job spread over all XCDs (few jobs, so latency, not key reuse
// through L2, is what matters).
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_term_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                    uint32_t L, const ModConst *__restrict__ mcs,
                                                                    const TwPair *__restrict__ tw) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, false>()];
    const uint32_t units = (L + 1) * L, jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const KsJob job = jobs[jb];
    const uint32_t jr = unit / L, i = unit % L;
    const uint32_t j = jr == 0 ? L : jr - 1;
    ks_stage_term<LOGN>(job.key, job.scratch, j, i, L, sh, mcs[j], tw);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_fold_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                    uint32_t L, const ModConst *__restrict__ mcs,
                                                                    const TwPair *__restrict__ itw) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN>()];
    const uint32_t units = 2 * (L + 1), jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const KsJob job = jobs[jb];
    const uint32_t jr = unit / 2, c = unit % 2;
    const uint32_t j = jr == 0 ? L : jr - 1;
    ks_stage_fold<LOGN>(job.scratch, j, c, L, sh, mcs[j], itw);
}

// Latency form, two kernels: terms straight from the input (digits folded
// in), then fold and mod-down together.  Grids are jobs x units with a job's
// units spread over all XCDs.
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_term_direct_kernel(const KsJob *__restrict__ jobs,
                                                                           uint32_t n, uint32_t L,
                                                                           const ModConst *__restrict__ mcs,
                                                                           const TwPair *__restrict__ tw,
                                                                           const TwPair *__restrict__ itw) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, false>()];
    const uint32_t units = (L + 1) * L, jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const KsJob job = jobs[jb];
    const uint32_t jr = unit / L, i = unit % L;
    const uint32_t j = jr == 0 ? L : jr - 1;
    ks_stage_term_direct<LOGN>(job.x, job.galois, job.key, job.scratch, j, i, L, sh, mcs[i], mcs[j], tw, itw);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_fold_moddown_kernel(const KsJob *__restrict__ jobs,
                                                                            uint32_t n, uint32_t L,
                                                                            const ModConst *__restrict__ mcs,
                                                                            const TwPair *__restrict__ tw,
                                                                            const TwPair *__restrict__ itw,
                                                                            const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN>()];
    const uint32_t units = 2 * L, jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const KsJob job = jobs[jb];
    const uint32_t j = unit % L, c = unit / L;
    ks_stage_fold_moddown<LOGN>(job.scratch, j, c, L, c == 0 ? job.add0 : job.add1, c == 0 ? job.galois : 0u,
                                job.addct, job.out, sh, mcs[j], mcs[L], tw, itw, mrc);
}

// Hoisted rotations (see ks_stage_hoisted_inner).  Mod-up: one workgroup per
// (source, modulus j, digit i), units with i == j exit at once; grid = jobs x
// units so one source spreads over all XCDs.
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_modup_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                     uint32_t L, const ModConst *__restrict__ mcs,
                                                                     const TwPair *__restrict__ tw) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, false>()];
    const uint32_t units = (L + 1) * L, jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const uint32_t jr = unit / L, i = unit % L;
    const uint32_t j = jr == 0 ? L : jr - 1;
    if (i == j) return;   // c1's own limb, used as is
    ks_stage_modup<LOGN>(jobs[jb].scratch, j, i, sh, mcs[j], tw, L);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_hoisted_inner_kernel(
    const KsJob *__restrict__ jobs, uint32_t n, uint32_t L, const ModConst *__restrict__ mcs,
    const TwPair *__restrict__ itw) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, false>()];
    const JobUnit ju = xcd_job_unit(blockIdx.x, L + 1, n);
    if (ju.job >= n) return;
    const KsJob job = jobs[ju.job];
    const uint32_t j = ju.unit == 0 ? L : ju.unit - 1;
    ks_stage_hoisted_inner<LOGN>(job.key, job.x, job.hoist, job.scratch, job.galois, j, L, sh, mcs[j], itw);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_moddown_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                       uint32_t L, const ModConst *__restrict__ mcs,
                                                                       const TwPair *__restrict__ tw,
                                                                       const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN>()];
    const JobUnit ju = xcd_job_unit(blockIdx.x, 2 * L, n);
    if (ju.job >= n) return;
    const KsJob job = jobs[ju.job];
    const uint32_t j = ju.unit % L, c = ju.unit / L;
    ks_stage_moddown<LOGN>(job.scratch, j, c, L, c == 0 ? job.add0 : job.add1, c == 0 ? job.galois : 0u,
                           job.addct, job.out, sh, mcs[j], tw, mrc, mcs[L].q);
}

size_t ks_scratch_words(const lola_ctx *ctx) { return (size_t)(4 * ctx->L + 2) * ctx->N; }

// Launches of at most this many jobs take the latency form of the inner
// stage (ks_term + ks_fold): L (L+1) workgroups per job instead of L+1, each
// one transform deep instead of L, at the price of 2 L (L+1) N more scratch
// words per job.
static constexpr uint32_t KS_TERM_MAX_JOBS = 16;
static bool ks_term_mode(uint32_t n) { return n <= KS_TERM_MAX_JOBS; }
// Within the latency form: terms straight from the input (two kernels) while
// they fit one round of workgroups over the CUs; beyond it the digit
// transforms each target repeats cost more than the two launches they save.
static bool ks_direct_mode(uint32_t n, uint32_t L) { return n * L * (L + 1) <= 256; }
static size_t ks_job_words(const lola_ctx *ctx, uint32_t n) {
    const size_t L = ctx->L;
    return ks_scratch_words(ctx) + (ks_term_mode(n) ? 2 * L * (L + 1) * ctx->N : 0);
}
size_t ks_launch_words(const lola_ctx *ctx, uint32_t n) { return (size_t)n * ks_job_words(ctx, n); }
size_t ks_chunk_words(const lola_ctx *ctx, uint32_t chunk) {
    return std::max(ks_launch_words(ctx, chunk), ks_launch_words(ctx, std::min(chunk, KS_TERM_MAX_JOBS)));
}

// Algorithmic cost of each key-switch kernel per launch of n jobs (bytes,
// lane-ops), with T the lane-ops of one limb transform:
//   digits       per (job, digit): reads x_i, writes X'_i and D_i: 12N B; one INTT
//   inner        per job: key 2L(L+1)N words, D and X' 2LN, U 2LN + 2N out;
//                L^2 + 2 transforms and 2L(L+1)N multiply-accumulates
//   moddown      per (job, prime, component): U, u_P, addend in, result out:
//                16N B; one NTT and ~10 ops a coefficient
//   term         per job: L(L+1) units, each a digit limb and two key limbs in,
//                two terms out (20N B); L^2 transforms, 2L(L+1)N products
//   fold         per job: 2(L+1) units, each L terms in and one limb out; the
//                special prime's two also INTT
//   term_direct  as term, plus each unit's digit INTT (i != j): 2 L^2 transforms
//   fold_moddown per job: 2L units, each the 2L terms of its prime and of P and
//                the addend in, one limb out; two transforms each
//   modup        per source: L^2 units (i != j), each one limb in and out, one NTT
//   hoisted      per rotation: key, the source's L(L+1) transformed digit limbs,
//                U and u_P out; two INTTs and the multiply-accumulates
// Bytes count each distinct key (2L(L+1)N words) and hoisting source's
// transformed digits (L(L+1)N words) once per launch: jobs that share them
// read them from HBM once.
struct KsCost {
    double N, L, T;
    explicit KsCost(const lola_ctx *ctx) : N(ctx->N), L(ctx->L), T(xform_ops(ctx)) {}
    double key_b() const { return 8 * N * L * (L + 1); }
    double digits_b() const { return 12 * N; }
    double inner_b(double n, double keys) const { return keys * key_b() + n * 8 * N * (2 * L + 1); }
    double inner_o() const { return (L * L + 2) * T + 2 * COST_MAC * L * (L + 1) * N; }
    double moddown_b() const { return 16 * N; }
    double moddown_o() const { return T + 10 * N; }
    double term_b() const { return 20 * N * L * (L + 1); }
    double term_o() const { return L * L * T + 2 * COST_MUL * L * (L + 1) * N; }
    double fold_b() const { return 8 * N * (L + 1) * (L + 1); }
    double fold_o() const { return 2 * T + 2 * (L + 1) * L * N * COST_ADD; }
    double direct_o() const { return 2 * L * L * T + 2 * COST_MUL * L * (L + 1) * N; }
    double foldmd_b() const { return 16 * N * L * (L + 1); }
    double foldmd_o() const { return 2 * L * (2 * T + 2 * L * N * COST_ADD + 10 * N); }
    double modup_b() const { return 8 * N * L * L; }
    double modup_o() const { return L * L * T; }
    double hoist_b(double n, double keys, double srcs) const {
        return keys * key_b() + srcs * 4 * N * L * (L + 1) + n * 8 * N * (L + 1);
    }
    double hoist_o() const { return 2 * T + 2 * COST_MAC * L * (L + 1) * N; }
};

int launch_keyswitch(lola_ctx *ctx, const KsJob *d_jobs, uint32_t n, const uint64_t *aux, hipStream_t s) {
    if (n == 0) return LOLA_OK;
    const uint32_t L = ctx->L;
    const dim3 block(ctx->N / NTT_E);
    const KsCost c(ctx);
    if (ctx->timing) ctx->timed_jobs += n;
    const bool term = ks_term_mode(n), direct = term && ks_direct_mode(n, L);
#define LOLA_KS_CASE(LG)                                                                                     \
    case LG:                                                                                                 \
        if (direct) {                                                                                        \
            LOLA_TIMED(ctx, s, KID_KS_TERM_DIRECT, n, c.term_b() * n, c.direct_o() * n,                       \
                       hipLaunchKernelGGL(ks_term_direct_kernel<LG>, dim3(n * (L + 1) * L), block, 0, s, d_jobs, \
                                          n, L, ctx->d_mc, ctx->d_tw, ctx->d_itw));                           \
            LOLA_TIMED(ctx, s, KID_KS_FOLD_MODDOWN, n, c.foldmd_b() * n, c.foldmd_o() * n,                    \
                       hipLaunchKernelGGL(ks_fold_moddown_kernel<LG>, dim3(n * 2 * L), block, 0, s, d_jobs, n, \
                                          L, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc));                  \
            break;                                                                                           \
        }                                                                                                    \
        LOLA_TIMED(ctx, s, KID_KS_DIGITS, n * L, c.digits_b() * n * L, c.T * n * L,                           \
                   hipLaunchKernelGGL(ks_digits_kernel<LG>, dim3(xcd_grid(n, L)), block, 0, s, d_jobs, n, L,    \
                                      ctx->d_mc, ctx->d_itw));                                                \
        if (term) {                                                                                          \
            LOLA_TIMED(ctx, s, KID_KS_TERM, n, c.term_b() * n, c.term_o() * n,                                \
                       hipLaunchKernelGGL(ks_term_kernel<LG>, dim3(n * (L + 1) * L), block, 0, s, d_jobs, n, L, \
                                          ctx->d_mc, ctx->d_tw));                                             \
            LOLA_TIMED(ctx, s, KID_KS_FOLD, n, c.fold_b() * n, c.fold_o() * n,                                \
                       hipLaunchKernelGGL(ks_fold_kernel<LG>, dim3(n * 2 * (L + 1)), block, 0, s, d_jobs, n, L, \
                                          ctx->d_mc, ctx->d_itw));                                            \
        } else {                                                                                             \
            LOLA_TIMED(ctx, s, KID_KS_INNER, n, c.inner_b(n, (double)aux[0]), c.inner_o() * n,                             \
                       hipLaunchKernelGGL(ks_inner_kernel<LG>, dim3(xcd_grid(n, L + 1)), block, 0, s, d_jobs, n, \
                                          L, ctx->d_mc, ctx->d_tw, ctx->d_itw));                              \
        }                                                                                                    \
        LOLA_TIMED(ctx, s, KID_KS_MODDOWN, n * 2 * L, c.moddown_b() * n * 2 * L, c.moddown_o() * n * 2 * L,    \
                   hipLaunchKernelGGL(ks_moddown_kernel<LG>, dim3(xcd_grid(n, 2 * L)), block, 0, s, d_jobs, n, \
                                      L, ctx->d_mc, ctx->d_tw, ctx->d_mrc));                                  \
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

int launch_keyswitch_hoist_src(lola_ctx *ctx, const KsJob *d_jobs, uint32_t n, hipStream_t s) {
    if (n == 0) return LOLA_OK;
    const uint32_t L = ctx->L;
    const dim3 block(ctx->N / NTT_E);
    const KsCost c(ctx);
#define LOLA_HS_CASE(LG)                                                                                     \
    case LG:                                                                                                 \
        LOLA_TIMED(ctx, s, KID_KS_HOIST_DIGITS, n * L, c.digits_b() * n * L, c.T * n * L,                           \
                   hipLaunchKernelGGL(ks_digits_kernel<LG>, dim3(xcd_grid(n, L)), block, 0, s, d_jobs, n, L,    \
                                      ctx->d_mc, ctx->d_itw));                                                \
        LOLA_TIMED(ctx, s, KID_KS_MODUP, n, c.modup_b() * n, c.modup_o() * n,                                 \
                   hipLaunchKernelGGL(ks_modup_kernel<LG>, dim3(n * (L + 1) * L), block, 0, s, d_jobs, n, L,    \
                                      ctx->d_mc, ctx->d_tw));                                                 \
        break;
    switch (ctx->logN) {
        LOLA_HS_CASE(10)
        LOLA_HS_CASE(11)
        LOLA_HS_CASE(12)
        LOLA_HS_CASE(13)
        LOLA_HS_CASE(14)
        default: return set_error(LOLA_E_PARAMS, "unsupported N");
    }
#undef LOLA_HS_CASE
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

int launch_keyswitch_hoist_rot(lola_ctx *ctx, const KsJob *d_jobs, uint32_t n, const uint64_t *aux,
                               hipStream_t s) {
    if (n == 0) return LOLA_OK;
    const uint32_t L = ctx->L;
    const dim3 block(ctx->N / NTT_E);
    const KsCost c(ctx);
#define LOLA_HR_CASE(LG)                                                                                     \
    case LG:                                                                                                 \
        LOLA_TIMED(ctx, s, KID_KS_HOISTED_INNER, n, c.hoist_b(n, (double)aux[0], (double)aux[1]), c.hoist_o() * n, \
                   hipLaunchKernelGGL(ks_hoisted_inner_kernel<LG>, dim3(xcd_grid(n, L + 1)), block, 0, s, d_jobs, \
                                      n, L, ctx->d_mc, ctx->d_itw));                                          \
        LOLA_TIMED(ctx, s, KID_KS_HOIST_MODDOWN, n * 2 * L, c.moddown_b() * n * 2 * L, c.moddown_o() * n * 2 * L,    \
                   hipLaunchKernelGGL(ks_moddown_kernel<LG>, dim3(xcd_grid(n, 2 * L)), block, 0, s, d_jobs, n, \
                                      L, ctx->d_mc, ctx->d_tw, ctx->d_mrc));                                  \
        break;
    switch (ctx->logN) {
        LOLA_HR_CASE(10)
        LOLA_HR_CASE(11)
        LOLA_HR_CASE(12)
        LOLA_HR_CASE(13)
        LOLA_HR_CASE(14)
        default: return set_error(LOLA_E_PARAMS, "unsupported N");
    }
#undef LOLA_HR_CASE
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

size_t ks_hoist_words(const lola_ctx *ctx) { return ks_hoist_limbs(ctx->L) * ctx->N; }

// Jobs per launch: bounds the scratch arena ((4L+2) N words per job).
static constexpr uint32_t KS_CHUNK = 128;

void program_keyswitch(const lola_ctx *ctx, Program &p, std::vector<KsJob> jobs, uint32_t *scratch,
                       uint32_t chunk, LaunchKind kind) {
    // jobs that share a key side by side (see xcd_job_unit); the order of the
    // jobs of one launch does not change any result
    std::stable_sort(jobs.begin(), jobs.end(), [](const KsJob &a, const KsJob &b) { return a.key < b.key; });
    for (size_t off = 0; off < jobs.size(); off += chunk) {
        const size_t n = std::min<size_t>(chunk, jobs.size() - off);
        // fits in ks_chunk_words(ctx, chunk); hoisted rotations take the
        // batched form whatever their number
        const size_t per = kind == LK_KS ? ks_job_words(ctx, (uint32_t)n) : ks_scratch_words(ctx);
        std::vector<KsJob> part(jobs.begin() + off, jobs.begin() + off + n);
        for (size_t k = 0; k < n; ++k) part[k].scratch = scratch + per * k;
        p.launch(kind, part);
        p.ks_jobs += n;
    }
}

int keyswitch_host_jobs(lola_ctx *ctx, std::vector<KsJob> &jobs, hipStream_t s) {
    for (size_t off = 0; off < jobs.size(); off += KS_CHUNK) {
        const uint32_t n = (uint32_t)std::min<size_t>(KS_CHUNK, jobs.size() - off);
        void *buf = nullptr;
        int rc = scratch_get(ctx, ks_launch_words(ctx, n) * 4, &buf);
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
    const uint32_t n = std::min<uint32_t>(std::max<uint32_t>(n_ct, 1), KS_CHUNK);
    return scratch_get(ctx, std::max(ks_chunk_words(ctx, n), n * mul_scratch_words(ctx)) * 4, &buf);
}

int lola_rotate_hoisted(lola_ctx *ctx, const uint32_t *in_dev, uint32_t n, const uint32_t *galois,
                        const uint32_t *const *keys, uint32_t *const *out_dev, lola_stream stream) {
    if (!ctx || (n && (!in_dev || !galois || !keys || !out_dev))) return set_error(LOLA_E_INVAL, "null argument");
    if (n == 0) return LOLA_OK;
    const size_t P = (size_t)ctx->L * ctx->N;
    for (uint32_t k = 0; k < n; ++k) {
        if (!keys[k]) return set_error(LOLA_E_NOKEY, "hoisted rotation without key");
        if (!out_dev[k]) return set_error(LOLA_E_INVAL, "null output ciphertext");
        if (out_dev[k] == in_dev) return set_error(LOLA_E_INVAL, "output aliases the input");
        if (galois[k] < 3 || !(galois[k] & 1) || galois[k] >= 2 * ctx->N)
            return set_error(LOLA_E_INVAL, "bad Galois element");
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t per = ks_scratch_words(ctx), hw = ks_hoist_words(ctx);
    for (uint32_t off = 0; off < n; off += KS_CHUNK) {
        const uint32_t m = std::min<uint32_t>(KS_CHUNK, n - off);
        void *buf = nullptr;
        int rc = scratch_get(ctx, (hw + per * m) * 4, &buf);
        if (rc) return rc;
        uint32_t *hoist = (uint32_t *)buf, *scr = hoist + hw;
        std::vector<KsJob> src{KsJob{in_dev + P, nullptr, nullptr, nullptr, nullptr, nullptr, hoist, 1, 0, nullptr}};
        std::vector<KsJob> rot(m);
        for (uint32_t k = 0; k < m; ++k)
            rot[k] = KsJob{in_dev + P, keys[off + k], in_dev, nullptr, nullptr, out_dev[off + k], scr + per * k,
                           galois[off + k], 0, hoist};
        Program p;
        p.launch(LK_KS_HSRC, src);
        p.launch(LK_KS_HROT, rot);
        if ((rc = program_run_now(ctx, p, s))) return rc;
    }
    return LOLA_OK;
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
