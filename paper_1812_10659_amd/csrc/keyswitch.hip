// Key switching (relinearisation and Galois rotations), batched over jobs.
//
// Three launches per batch, one workgroup per limb-sized unit of work (the
// stages themselves are in ks_core.hpp):
//   ks_digits   (L per job):    gather sigma_g(x_i) (kept), INTT -> x_i in coefficients
//   ks_inner    (L+K per job):  for target modulus m_j: for each digit d,
//                               its value mod m_j (Garner for a digit of two
//                               primes), NTT (a digit holding q_j reuses
//                               x_j), multiply-accumulate with the key; for a
//                               special prime the two sums are also brought
//                               back to coefficients
//   ks_moddown  (2L per job):   lift [u_P]_P into q_j, NTT, subtract, times
//                               P^-1, add the c0 (or d0 / d1) term and an
//                               optional whole-ciphertext addend (fused
//                               rotate-and-add).
#include <algorithm>
#include <cstring>

#include "ks_core.hpp"
#include "program.hpp"

namespace lola {

// Stage kernels are compiled in several radix splits and LDS placements
// (the key-switch autotuner's variants, below); SPLIT 0 is the default
// grouping of stages into passes.
template <int LOGN, int SPLIT = 0, bool PAD = true>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_digits_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                      uint32_t L, const ModConst *__restrict__ mcs,
                                                                      const TwPair *__restrict__ itw, uint32_t keep) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, PAD>()];
    const JobUnit ju = xcd_job_unit(blockIdx.x, L, n);
    if (ju.job >= n) return;
    const KsJob job = jobs[ju.job];
    const uint32_t i = ju.unit;
    ks_stage_digit<LOGN, PAD, SPLIT>(job.x, job.galois, job.scratch, i, L, sh, mcs[i], itw, keep != 0);
}

// Target modulus of unit u of a job whose first K units are the special
// primes' (p_u), the others q_0..q_{L-1}.
__device__ __forceinline__ uint32_t ks_unit_modulus(const KsDims &kd, uint32_t u) {
    return u < kd.K ? kd.L + u : u - kd.K;
}

template <int LOGN, int KSI = ks_inner_split<LOGN>(), bool LAZY = false>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_inner_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                     const KsDims kd,
                                                                     const ModConst *__restrict__ mcs,
                                                                     const TwPair *__restrict__ tw,
                                                                     const TwPair *__restrict__ itw,
                                                                     const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[2 << LOGN];   // two halves for the plain placement
    // target modulus: q_j (j < L) or p_k (j = L + k); the special primes'
    // units, longer than the others by their two inverse transforms, are
    // dispatched ahead of the XCD's other units so the launch's tail holds
    // short ones
    const JobUnit ju = xcd_job_unit_lead(blockIdx.x, kd.M(), kd.K, n);
    if (ju.job >= n) return;
    const KsJob job = jobs[ju.job];
    const uint32_t j = ks_unit_modulus(kd, ju.unit);
    ks_stage_inner<LOGN, KSI, (1u << LOGN), 0, LAZY, true>(job.key, job.scratch, j, kd, sh, mcs[j], tw, itw, mrc,
                                                             job.x, job.galois);
}

// Latency form of the inner stage (launches of at most KS_TERM_MAX_JOBS
// jobs): (L+K) dn workgroups per job, one digit term each, then 2 (L+K) that
// fold the terms.  The special primes' units come first, as above.  Grid =
// jobs x units, workgroup k taking unit k mod units of job k / units: the
// units of one job spread over all XCDs (few jobs, so latency, not key reuse
// through L2, is what matters).
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_term_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                    const KsDims kd,
                                                                    const ModConst *__restrict__ mcs,
                                                                    const TwPair *__restrict__ tw,
                                                                    const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, false>()];
    const uint32_t units = kd.M() * kd.dn, jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const KsJob job = jobs[jb];
    const uint32_t j = ks_unit_modulus(kd, unit / kd.dn), d = unit % kd.dn;
    ks_stage_term<LOGN>(job.key, job.scratch, j, d, kd, sh, mcs[j], tw, mrc);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_fold_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                    const KsDims kd,
                                                                    const ModConst *__restrict__ mcs,
                                                                    const TwPair *__restrict__ itw) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN>()];
    const uint32_t units = 2 * kd.M(), jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const KsJob job = jobs[jb];
    const uint32_t j = ks_unit_modulus(kd, unit / 2), c = unit % 2;
    ks_stage_fold<LOGN>(job.scratch, j, c, kd, sh, mcs[j], itw);
}

// Latency form, two kernels: terms straight from the input (digits folded
// in), then fold and mod-down together.  Grids are jobs x units with a job's
// units spread over all XCDs.
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_term_direct_kernel(const KsJob *__restrict__ jobs,
                                                                           uint32_t n, const KsDims kd,
                                                                           const ModConst *__restrict__ mcs,
                                                                           const TwPair *__restrict__ tw,
                                                                           const TwPair *__restrict__ itw,
                                                                           const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, false>()];
    const uint32_t units = kd.M() * kd.dn, jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const KsJob job = jobs[jb];
    const uint32_t j = ks_unit_modulus(kd, unit / kd.dn), d = unit % kd.dn;
    ks_stage_term_direct<LOGN>(job.x, job.galois, job.key, job.scratch, j, d, kd, sh, mcs, tw, itw, mrc);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_fold_moddown_kernel(const KsJob *__restrict__ jobs,
                                                                            uint32_t n, const KsDims kd,
                                                                            const ModConst *__restrict__ mcs,
                                                                            const TwPair *__restrict__ tw,
                                                                            const TwPair *__restrict__ itw,
                                                                            const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN>()];
    const uint32_t L = kd.L, units = 2 * L, jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const KsJob job = jobs[jb];
    const uint32_t j = unit % L, c = unit / L;
    ks_stage_fold_moddown<LOGN>(job.scratch, j, c, kd, c == 0 ? job.add0 : job.add1, c == 0 ? job.galois : 0u,
                                job.addct, job.out, sh, mcs, tw, itw, mrc);
}

// Hoisted rotations (see ks_stage_hoisted_inner).  Mod-up: one workgroup per
// (source, modulus j, digit d), units whose digit holds q_j exit at once;
// grid = jobs x units so one source spreads over all XCDs.
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_modup_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                     const KsDims kd,
                                                                     const ModConst *__restrict__ mcs,
                                                                     const TwPair *__restrict__ tw,
                                                                     const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, false>()];
    const uint32_t units = kd.M() * kd.dn, jb = blockIdx.x / units, unit = blockIdx.x % units;
    if (jb >= n) return;
    const uint32_t j = ks_unit_modulus(kd, unit / kd.dn), d = unit % kd.dn;
    if (kd.owns(d, j)) return;   // c1's own limb, used as is
    ks_stage_modup<LOGN>(jobs[jb].scratch, j, d, sh, mcs[j], tw, kd, mrc);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_hoisted_inner_kernel(
    const KsJob *__restrict__ jobs, uint32_t n, const KsDims kd, const ModConst *__restrict__ mcs,
    const TwPair *__restrict__ itw) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, false>()];
    // L + 2K units per job: the special primes' two each (one per key
    // component, each with an inverse transform, so the longest) ahead of the
    // XCD's other units, then q_0..q_{L-1}
    const uint32_t lead = 2 * kd.K;
    const JobUnit ju = xcd_job_unit_lead(blockIdx.x, kd.L + lead, lead, n);
    if (ju.job >= n) return;
    const KsJob job = jobs[ju.job];
    const uint32_t j = ju.unit < lead ? kd.L + ju.unit / 2 : ju.unit - lead, c = ju.unit < lead ? ju.unit % 2 : 0;
    ks_stage_hoisted_inner<LOGN>(job.key, job.x, job.hoist, job.scratch, job.galois, j, c, kd, sh, mcs[j], itw);
}

template <int LOGN, int SPLIT = 0, bool PAD = true>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks_moddown_kernel(const KsJob *__restrict__ jobs, uint32_t n,
                                                                       const KsDims kd,
                                                                       const ModConst *__restrict__ mcs,
                                                                       const TwPair *__restrict__ tw,
                                                                       const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN, PAD>()];
    const uint32_t L = kd.L;
    const JobUnit ju = xcd_job_unit(blockIdx.x, 2 * L, n);
    if (ju.job >= n) return;
    const KsJob job = jobs[ju.job];
    const uint32_t j = ju.unit % L, c = ju.unit / L;
    ks_stage_moddown<LOGN, PAD, SPLIT>(job.scratch, j, c, kd, c == 0 ? job.add0 : job.add1, c == 0 ? job.galois : 0u,
                                       job.addct, job.out, sh, mcs[j], tw, mrc, mcs[L].q);
}

// ---- stage variants (radix split x LDS placement) and their launchers ----
// At N = 16384 each batched stage is compiled in a few variants; the
// context's ks_var[stage] picks one (0 = default).  Every variant computes
// the same words; lola_ks_autotune times them and keeps the fastest.
struct KsStageVariant {
    uint32_t split, padded;
};
static const KsStageVariant KS_VARIANTS[3][4] = {
    {{4442, 1}, {4442, 0}, {4433, 1}, {4244, 1}},   // digits
    {{4433, 0}, {4442, 0}, {4424, 0}, {0, 0}},      // inner (plain placement, two LDS halves)
    {{4442, 1}, {4442, 0}, {4433, 1}, {4244, 1}}};  // mod-down
static uint32_t ks_variant_count(uint32_t logN, uint32_t stage) {
    if (logN != 14 || stage > 2) return 1;
    return stage == 1 ? 3 : 4;
}

// keep: also store sigma_g(x_i) (needed by the term form only; the inner
// kernel reads it from the input, and hoisted sources never use it).
template <int LG>
static void launch_ks_digits(lola_ctx *ctx, const KsJob *d, uint32_t n, bool keep, hipStream_t s) {
    const uint32_t L = ctx->L, k = keep ? 1u : 0u;
    const dim3 g(xcd_grid(n, L)), b(ctx->N / NTT_E);
    if constexpr (LG == 14) {
        switch (ctx->ks_var[0]) {
            case 1: hipLaunchKernelGGL((ks_digits_kernel<14, 0, false>), g, b, 0, s, d, n, L, ctx->d_mc, ctx->d_itw, k); return;
            case 2: hipLaunchKernelGGL((ks_digits_kernel<14, 4433, true>), g, b, 0, s, d, n, L, ctx->d_mc, ctx->d_itw, k); return;
            case 3: hipLaunchKernelGGL((ks_digits_kernel<14, 4244, true>), g, b, 0, s, d, n, L, ctx->d_mc, ctx->d_itw, k); return;
            default: break;
        }
    }
    hipLaunchKernelGGL((ks_digits_kernel<LG, 0, true>), g, b, 0, s, d, n, L, ctx->d_mc, ctx->d_itw, k);
}

template <int LG>
static void launch_ks_inner(lola_ctx *ctx, const KsJob *d, uint32_t n, hipStream_t s) {
    const KsDims kd = ks_dims(ctx);
    const dim3 g(xcd_grid(n, kd.M())), b(ctx->N / NTT_E);
    if constexpr (LG == 14) {
        // at most four digits: the transforms' outputs enter the 64-bit sums
        // unreduced (see ks_stage_inner)
        if (kd.dn <= 4) {
            switch (ctx->ks_var[1]) {
                case 1: hipLaunchKernelGGL((ks_inner_kernel<14, 0, true>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc); return;
                case 2: hipLaunchKernelGGL((ks_inner_kernel<14, 4424, true>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc); return;
                default: hipLaunchKernelGGL((ks_inner_kernel<14, 4433, true>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc); return;
            }
        }
        switch (ctx->ks_var[1]) {
            case 1: hipLaunchKernelGGL((ks_inner_kernel<14, 0>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc); return;
            case 2: hipLaunchKernelGGL((ks_inner_kernel<14, 4424>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc); return;
            default: break;
        }
    }
    hipLaunchKernelGGL((ks_inner_kernel<LG>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc);
}

template <int LG>
static void launch_ks_moddown(lola_ctx *ctx, const KsJob *d, uint32_t n, hipStream_t s) {
    const KsDims kd = ks_dims(ctx);
    const dim3 g(xcd_grid(n, 2 * kd.L)), b(ctx->N / NTT_E);
    if constexpr (LG == 14) {
        switch (ctx->ks_var[2]) {
            case 1: hipLaunchKernelGGL((ks_moddown_kernel<14, 0, false>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_mrc); return;
            case 2: hipLaunchKernelGGL((ks_moddown_kernel<14, 4433, true>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_mrc); return;
            case 3: hipLaunchKernelGGL((ks_moddown_kernel<14, 4244, true>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_mrc); return;
            default: break;
        }
    }
    hipLaunchKernelGGL((ks_moddown_kernel<LG, 0, true>), g, b, 0, s, d, n, kd, ctx->d_mc, ctx->d_tw, ctx->d_mrc);
}

size_t ks_scratch_words(const lola_ctx *ctx) { return (size_t)(4 * ctx->L + 2 * ctx->K) * ctx->N; }

// Autotuning inputs: pseudo-random words below `bound` (every modulus of the
// context exceeds it, so each word is a valid residue in any limb).
__global__ void ks_tune_fill_kernel(uint32_t *x, size_t nx, uint32_t *k, size_t nk, uint32_t bound) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx + nk) return;
    uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    const uint32_t v = (uint32_t)(h % bound);
    if (i < nx) x[i] = v;
    else k[i - nx] = v;
}

// Launches of at most this many jobs take the latency form of the inner
// stage (ks_term + ks_fold): (L+K) dn workgroups per job instead of L+K, each
// one transform deep instead of dn, at the price of 2 (L+K) dn N more
// scratch words per job.
static constexpr uint32_t KS_TERM_MAX_JOBS = 16;
static bool ks_term_mode(uint32_t n) { return n <= KS_TERM_MAX_JOBS; }
// Within the latency form: terms straight from the input (two kernels) while
// they fit one round of workgroups over the CUs; beyond it the digit
// transforms each target repeats cost more than the two launches they save.
// Only with one prime per digit: a digit of two primes makes each of the two
// kernels three transforms deep (two inverse transforms before the term's
// transform, two special primes' before the mod-down's), against one per
// kernel in the four-kernel form.
static bool ks_direct_mode(uint32_t n, const KsDims &kd) { return kd.K == 1 && n * kd.dn * kd.M() <= 256; }
static size_t ks_job_words(const lola_ctx *ctx, uint32_t n) {
    const KsDims kd = ks_dims(ctx);
    return ks_scratch_words(ctx) + (ks_term_mode(n) ? 2 * (size_t)kd.M() * kd.dn * ctx->N : 0);
}
size_t ks_launch_words(const lola_ctx *ctx, uint32_t n) { return (size_t)n * ks_job_words(ctx, n); }
size_t ks_chunk_words(const lola_ctx *ctx, uint32_t chunk) {
    return std::max(ks_launch_words(ctx, chunk), ks_launch_words(ctx, std::min(chunk, KS_TERM_MAX_JOBS)));
}

// Algorithmic cost of each key-switch kernel per launch of n jobs (bytes,
// lane-ops), with T the lane-ops of one limb transform, M = L + K target
// moduli, dn digits, X = dn M - L the (target, digit) pairs that need a
// transform (a digit holding the target reuses x_j), and G the pairs whose
// digit has two primes (a Garner step per coefficient, COST_GARNER):
//   digits       per (job, prime): reads x_i, writes X'_i and x_i: 12N B; one INTT
//   inner        per job: key 2 dn M N words, x and X' 2LN, U 2LN + 2KN out;
//                X + 2K transforms and 2 dn M N multiply-accumulates
//   moddown      per (job, prime, component): U, u_P, addend in, result out:
//                16N B (20N with two special primes); one NTT and ~10 ops a
//                coefficient (plus a Garner step with two special primes)
//   term         per job: dn M units, each a digit's limbs and two key limbs
//                in, two terms out; X transforms, 2 dn M N products
//   fold         per job: 2M units, each dn terms in and one limb out; the
//                special primes' also INTT
//   term_direct  as term, plus each unit's digit INTTs (one per prime of the
//                digit, unless the digit holds the target)
//   fold_moddown per job: 2L units, each the dn terms of its prime and of every
//                special prime and the addend in, one limb out; K + 1 transforms
//   modup        per source: X units, each the digit's limbs in and one out, one NTT
//   hoisted      per rotation: key, the source's dn M transformed digit limbs,
//                U and u_P out; 2K INTTs and the multiply-accumulates
// Bytes count each distinct key (2 dn M N words) and hoisting source's
// transformed digits (dn M N words) once per launch: jobs that share them
// read them from HBM once.
struct KsCost {
    double N, L, K, M, dn, T, X, G, W;
    explicit KsCost(const lola_ctx *ctx) : N(ctx->N), L(ctx->L), K(ctx->K), T(xform_ops(ctx)) {
        const KsDims kd = ks_dims(ctx);
        M = kd.M();
        dn = kd.dn;
        X = dn * M - L;
        G = 0;
        W = 0;   // digit-limb INTTs of the direct form's units
        for (uint32_t d = 0; d < kd.dn; ++d) {
            const double own = kd.width(d), tgt = M - own;
            if (kd.width(d) == 2) G += tgt;
            W += tgt * own;
        }
    }
    double key_b() const { return 8 * N * dn * M; }
    double digits_b(bool keep) const { return (keep ? 12 : 8) * N; }
    double inner_b(double n, double keys) const { return keys * key_b() + n * 8 * N * (2 * L + K); }
    double inner_o() const { return (X + 2 * K) * T + 2 * COST_MAC * dn * M * N + G * N * COST_GARNER; }
    double moddown_b() const { return (12 + 4 * K) * N; }
    double moddown_o() const { return T + 10 * N + (K > 1 ? COST_GARNER * N : 0); }
    double term_b() const { return 20 * N * dn * M + 4 * N * G; }
    double term_o() const { return X * T + 2 * COST_MUL * dn * M * N + G * N * COST_GARNER; }
    double fold_b() const { return 8 * N * M * (dn + 1); }
    double fold_o() const { return 2 * K * T + 2 * M * dn * N * COST_ADD; }
    double direct_o() const { return (X + W) * T + 2 * COST_MUL * dn * M * N + G * N * COST_GARNER; }
    double foldmd_b() const { return 8 * N * L * ((K + 1) * dn + 2); }
    double foldmd_o() const {
        return 2 * L * ((K + 1) * T + (K + 1) * dn * N * COST_ADD + 10 * N + (K > 1 ? COST_GARNER * N : 0));
    }
    double modup_b() const { return 8 * N * X + 4 * N * G; }
    double modup_o() const { return X * T + G * N * COST_GARNER; }
    double hoist_b(double n, double keys, double srcs) const {
        return keys * key_b() + srcs * 4 * N * dn * M + n * 8 * N * (L + K);
    }
    double hoist_o() const { return 2 * K * T + 2 * COST_MAC * dn * M * N; }
};

double ks_whole_ops(const lola_ctx *ctx) {
    const KsCost c(ctx);
    return c.L * c.T + c.inner_o() + 2 * c.L * c.moddown_o();
}
double ks_whole_bytes(const lola_ctx *ctx) { return 4.0 * ctx->N * (4.0 * ctx->L + 2.0 * ctx->dnum() * (ctx->L + ctx->K)); }

int launch_keyswitch(lola_ctx *ctx, const KsJob *d_jobs, uint32_t n, const uint64_t *aux, hipStream_t s) {
    if (n == 0) return LOLA_OK;
    const uint32_t L = ctx->L;
    const KsDims kd = ks_dims(ctx);
    const uint32_t TU = kd.M() * kd.dn;   // term units per job
    const dim3 block(ctx->N / NTT_E);
    const KsCost c(ctx);
    if (ctx->timing) ctx->timed_jobs += n;
    const bool term = ks_term_mode(n), direct = term && ks_direct_mode(n, kd);
#define LOLA_KS_CASE(LG)                                                                                     \
    case LG:                                                                                                 \
        if (direct) {                                                                                        \
            LOLA_TIMED(ctx, s, KID_KS_TERM_DIRECT, n, c.term_b() * n, c.direct_o() * n,                       \
                       hipLaunchKernelGGL(ks_term_direct_kernel<LG>, dim3(n * TU), block, 0, s, d_jobs, n, kd,  \
                                          ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc));                     \
            LOLA_TIMED(ctx, s, KID_KS_FOLD_MODDOWN, n, c.foldmd_b() * n, c.foldmd_o() * n,                    \
                       hipLaunchKernelGGL(ks_fold_moddown_kernel<LG>, dim3(n * 2 * L), block, 0, s, d_jobs, n, \
                                          kd, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc));                 \
            break;                                                                                           \
        }                                                                                                    \
        LOLA_TIMED(ctx, s, KID_KS_DIGITS, n * L, c.digits_b(term) * n * L, c.T * n * L,                       \
                   launch_ks_digits<LG>(ctx, d_jobs, n, term, s));                                            \
        if (term) {                                                                                          \
            LOLA_TIMED(ctx, s, KID_KS_TERM, n, c.term_b() * n, c.term_o() * n,                                \
                       hipLaunchKernelGGL(ks_term_kernel<LG>, dim3(n * TU), block, 0, s, d_jobs, n, kd,         \
                                          ctx->d_mc, ctx->d_tw, ctx->d_mrc));                                 \
            LOLA_TIMED(ctx, s, KID_KS_FOLD, n, c.fold_b() * n, c.fold_o() * n,                                \
                       hipLaunchKernelGGL(ks_fold_kernel<LG>, dim3(n * 2 * kd.M()), block, 0, s, d_jobs, n, kd, \
                                          ctx->d_mc, ctx->d_itw));                                            \
        } else {                                                                                             \
            LOLA_TIMED(ctx, s, KID_KS_INNER, n, c.inner_b(n, (double)aux[0]), c.inner_o() * n,                 \
                       launch_ks_inner<LG>(ctx, d_jobs, n, s));                                               \
        }                                                                                                    \
        LOLA_TIMED(ctx, s, KID_KS_MODDOWN, n * 2 * L, c.moddown_b() * n * 2 * L, c.moddown_o() * n * 2 * L,    \
                   launch_ks_moddown<LG>(ctx, d_jobs, n, s));                                                 \
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
    const KsDims kd = ks_dims(ctx);
    const dim3 block(ctx->N / NTT_E);
    const KsCost c(ctx);
#define LOLA_HS_CASE(LG)                                                                                     \
    case LG:                                                                                                 \
        LOLA_TIMED(ctx, s, KID_KS_HOIST_DIGITS, n * L, c.digits_b(false) * n * L, c.T * n * L,                \
                   launch_ks_digits<LG>(ctx, d_jobs, n, false, s));                                           \
        LOLA_TIMED(ctx, s, KID_KS_MODUP, n, c.modup_b() * n, c.modup_o() * n,                                 \
                   hipLaunchKernelGGL(ks_modup_kernel<LG>, dim3(n * kd.M() * kd.dn), block, 0, s, d_jobs, n, kd, \
                                      ctx->d_mc, ctx->d_tw, ctx->d_mrc));                                     \
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
    const KsDims kd = ks_dims(ctx);
    const dim3 block(ctx->N / NTT_E);
    const KsCost c(ctx);
#define LOLA_HR_CASE(LG)                                                                                     \
    case LG:                                                                                                 \
        LOLA_TIMED(ctx, s, KID_KS_HOISTED_INNER, n, c.hoist_b(n, (double)aux[0], (double)aux[1]), c.hoist_o() * n, \
                   hipLaunchKernelGGL(ks_hoisted_inner_kernel<LG>, dim3(xcd_grid(n, L + 2 * kd.K)), block, 0, s,   \
                                      d_jobs, n, kd, ctx->d_mc, ctx->d_itw));                                 \
        LOLA_TIMED(ctx, s, KID_KS_HOIST_MODDOWN, n * 2 * L, c.moddown_b() * n * 2 * L, c.moddown_o() * n * 2 * L, \
                   launch_ks_moddown<LG>(ctx, d_jobs, n, s));                                                 \
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

size_t ks_hoist_words(const lola_ctx *ctx) { return ks_hoist_limbs(ks_dims(ctx)) * ctx->N; }

// Jobs per launch: bounds the scratch arena ((4L+2K) N words per job).
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

int lola_ks_variants(const lola_ctx *ctx, uint32_t stage, lola_ks_variant *out, uint32_t cap, uint32_t *count) {
    if (!ctx || !count || (cap && !out) || stage > 2) return set_error(LOLA_E_INVAL, "bad argument");
    const uint32_t nv = ks_variant_count(ctx->logN, stage);
    for (uint32_t v = 0; v < nv && v < cap; ++v) {
        const KsStageVariant &k = KS_VARIANTS[stage][v];
        out[v] = lola_ks_variant{stage, v, ctx->logN == 14 ? k.split : 0u, ctx->logN == 14 ? k.padded : 1u, 0.f};
    }
    *count = nv;
    return LOLA_OK;
}

int lola_ks_get_variant(const lola_ctx *ctx, uint32_t stage, uint32_t *index) {
    if (!ctx || !index || stage > 2) return set_error(LOLA_E_INVAL, "bad argument");
    *index = ctx->ks_var[stage];
    return LOLA_OK;
}

int lola_ks_set_variant(lola_ctx *ctx, uint32_t stage, uint32_t index) {
    if (!ctx || stage > 2) return set_error(LOLA_E_INVAL, "bad argument");
    if (index >= ks_variant_count(ctx->logN, stage)) return set_error(LOLA_E_INVAL, "no such key-switch variant");
    ctx->ks_var[stage] = index;
    return LOLA_OK;
}

int lola_ks_autotune(lola_ctx *ctx, uint32_t n_jobs, uint32_t reps, lola_ks_variant *out, uint32_t cap,
                     uint32_t *chosen, lola_stream stream) {
    if (!ctx || !chosen || (cap && !out) || n_jobs == 0 || n_jobs > KS_CHUNK || reps == 0)
        return set_error(LOLA_E_INVAL, "bad argument (1 <= n_jobs <= 128, reps >= 1)");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = ctx->N, L = ctx->L, ct = 2 * L * N, key = (size_t)ctx->dnum() * 2 * (L + ctx->K) * N;
    const size_t words = n_jobs * ct * 2 + key;   // inputs, outputs, one key
    const uint32_t saved[3] = {ctx->ks_var[0], ctx->ks_var[1], ctx->ks_var[2]};
    uint32_t *buf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto fail = [&](int rc) {
        if (buf) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(buf);
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (int k = 0; k < 3; ++k) ctx->ks_var[k] = saved[k];
        return rc;
    };
    if (hipMalloc(&buf, words * 4) != hipSuccess) return fail(set_error(LOLA_E_NOMEM, "autotune buffers"));
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(set_error(LOLA_E_DEVICE, "autotune events"));
    uint32_t *in = buf, *outb = buf + n_jobs * ct, *kd = buf + 2 * n_jobs * ct;
    // residues below every modulus of the context, so valid in each limb
    uint32_t bound = ctx->primes[0];
    for (uint32_t k = 0; k < ctx->L + ctx->K; ++k) bound = std::min(bound, ctx->primes[k]);
    hipLaunchKernelGGL(ks_tune_fill_kernel, dim3((unsigned)((n_jobs * ct + key + 255) / 256)), dim3(256), 0, s, in,
                       n_jobs * ct, kd, key, bound);
    // rotations by 3 (sigma_3), one key, as many jobs as given
    std::vector<KsJob> jobs(n_jobs);
    for (uint32_t k = 0; k < n_jobs; ++k)
        jobs[k] = KsJob{in + k * ct + L * N, kd, in + k * ct, nullptr, nullptr, outb + k * ct, nullptr, 3, 0};
    std::vector<uint32_t> ref(n_jobs * ct), got(n_jobs * ct);
    auto run = [&]() -> int {
        std::vector<KsJob> j = jobs;
        return keyswitch_host_jobs(ctx, j, s);
    };
    for (int k = 0; k < 3; ++k) ctx->ks_var[k] = 0;
    int rc = run();
    if (rc) return fail(rc);
    if (hipMemcpyAsync(ref.data(), outb, ref.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(set_error(LOLA_E_DEVICE, "autotune reference"));
    // stage by stage, the others at their best so far: every variant must
    // give the default's words before it is timed (the whole key switch,
    // reps times)
    uint32_t written = 0;
    for (uint32_t stage = 0; stage < 3; ++stage) {
        const uint32_t nv = ks_variant_count(ctx->logN, stage);
        float best_ms = 0;
        uint32_t best = 0;
        for (uint32_t v = 0; v < nv; ++v) {
            ctx->ks_var[stage] = v;
            if ((rc = run())) return fail(rc);
            if (hipMemcpyAsync(got.data(), outb, got.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(set_error(LOLA_E_DEVICE, "autotune readback"));
            if (memcmp(got.data(), ref.data(), got.size() * 4) != 0)
                return fail(set_error(LOLA_E_DEVICE, "autotune: key-switch stage " + std::to_string(stage) +
                                                         " variant " + std::to_string(v) + " differs from the default"));
            if (hipEventRecord(e0, s) != hipSuccess) return fail(set_error(LOLA_E_DEVICE, "autotune event"));
            for (uint32_t r = 0; r < reps; ++r)
                if ((rc = run())) return fail(rc);
            float t = 0;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess)
                return fail(set_error(LOLA_E_DEVICE, "autotune timing"));
            t /= (float)reps;
            // a variant replaces the best so far only when it is at least 1%
            // faster: closer figures are within the run-to-run spread, and the
            // default is what the other measurements were taken with
            if (v == 0 || t < best_ms * 0.99f) {
                best_ms = t;
                best = v;
            }
            if (written < cap) {
                const KsStageVariant &k = KS_VARIANTS[stage][v];
                out[written] = lola_ks_variant{stage, v, ctx->logN == 14 ? k.split : 0u,
                                               ctx->logN == 14 ? k.padded : 1u, t};
            }
            ++written;
        }
        ctx->ks_var[stage] = best;
        chosen[stage] = best;
    }
    const uint32_t picked[3] = {chosen[0], chosen[1], chosen[2]};
    fail(LOLA_OK);   // frees the buffers and restores the saved variants
    for (int k = 0; k < 3; ++k) ctx->ks_var[k] = picked[k];
    return written > cap ? set_error(LOLA_E_INVAL, "more variants than cap (all were timed and the best kept)")
                         : LOLA_OK;
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
