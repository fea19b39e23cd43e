// A rotation that allocates nothing: the same key switch as lola_rotate
// (digits, inner product, mod-down; the batched kernels' stage functions),
// with its scratch in a fixed device array instead of the context's arena,
// and its one job descriptor passed to each kernel by value instead of
// through the descriptor ring.  For callers that cannot allocate device
// memory (code under graph capture, tight serving loops).
//
// The array lives in this file's code object, once per GPU the library runs
// on, until the process ends.  Host code never uses its name as an address:
// each device's address comes from hipGetSymbolAddress, taken once per device
// with that device current (noalloc_setup, called by lola_ctx_create; the
// entry point calls it too, which returns at once once set up).
#include <mutex>

#include "ks_core.hpp"

namespace lola {

// One key switch's scratch, (4L + 2K) N words, at the largest L, K and N the
// library accepts: 52 x 16384 words = 3.25 MiB.
constexpr size_t NOALLOC_SCRATCH_WORDS = (size_t)(4 * MAXL + 2 * MAXK) * 16384;
static __device__ __align__(256) uint32_t scratch[NOALLOC_SCRATCH_WORDS];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_noalloc_mu;
static uint32_t *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

int noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return set_error(LOLA_E_INVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return LOLA_OK;
    int cur = 0;
    LOLA_HIP(hipGetDevice(&cur));
    LOLA_HIP(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return check_hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_noalloc_ptr[device] = (uint32_t *)p;
    return LOLA_OK;
}

// The batched stage kernels' bodies for a single job taken by value.
template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks1_digits_kernel(KsJob job, uint32_t L,
                                                                       const ModConst *__restrict__ mcs,
                                                                       const TwPair *__restrict__ itw) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN>()];
    const uint32_t i = blockIdx.x;
    ks_stage_digit<LOGN>(job.x, job.galois, job.scratch, i, L, sh, mcs[i], itw, false);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks1_inner_kernel(KsJob job, const KsDims kd,
                                                                      const ModConst *__restrict__ mcs,
                                                                      const TwPair *__restrict__ tw,
                                                                      const TwPair *__restrict__ itw,
                                                                      const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[2 << LOGN];
    // the special primes' units first
    const uint32_t j = blockIdx.x < kd.K ? kd.L + blockIdx.x : blockIdx.x - kd.K;
    ks_stage_inner<LOGN, ks_inner_split<LOGN>(), (1u << LOGN), 0, false, true>(job.key, job.scratch, j, kd, sh, mcs[j], tw,
                                                                              itw, mrc, job.x, job.galois);
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void ks1_moddown_kernel(KsJob job, const KsDims kd,
                                                                        const ModConst *__restrict__ mcs,
                                                                        const TwPair *__restrict__ tw,
                                                                        const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[ntt_lds_words<LOGN>()];
    const uint32_t L = kd.L, j = blockIdx.x % L, c = blockIdx.x / L;
    ks_stage_moddown<LOGN>(job.scratch, j, c, kd, c == 0 ? job.add0 : job.add1, c == 0 ? job.galois : 0u,
                           job.addct, job.out, sh, mcs[j], tw, mrc, mcs[L].q);
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_rotate_noalloc(lola_ctx *ctx, const uint32_t *gk, uint32_t galois, const uint32_t *ct, uint32_t *out,
                        lola_stream stream) {
    if (!ctx || !ct || !out) return set_error(LOLA_E_INVAL, "null argument");
    if (!gk) return set_error(LOLA_E_NOKEY, "missing Galois key");
    if (galois == 0 || !(galois & 1) || galois >= 2 * ctx->N) return set_error(LOLA_E_INVAL, "bad Galois element");
    if (out == ct) return set_error(LOLA_E_INVAL, "output aliases the input");
    const size_t words = (size_t)(4 * ctx->L + 2 * ctx->K) * ctx->N;
    if (words > NOALLOC_SCRATCH_WORDS)
        return set_error(LOLA_E_SHAPE, "key-switch scratch of " + std::to_string(words) +
                                           " words exceeds the fixed area of " +
                                           std::to_string(NOALLOC_SCRATCH_WORDS));
    // set up when the context was created; the first call on a device does it
    // otherwise (no allocation either way)
    int rc = noalloc_setup(ctx->device);
    if (rc) return rc;
    uint32_t *scr = g_noalloc_ptr[ctx->device];
    const size_t P = (size_t)ctx->L * ctx->N;
    const KsJob job{ct + P, gk, ct, nullptr, nullptr, out, scr, galois, 0, nullptr};
    hipStream_t s = (hipStream_t)stream;
    const uint32_t L = ctx->L;
    const KsDims kd = ks_dims(ctx);
    const dim3 block(ctx->N / NTT_E);
#define LOLA_KS1_CASE(LG)                                                                                    \
    case LG:                                                                                                 \
        hipLaunchKernelGGL(ks1_digits_kernel<LG>, dim3(L), block, 0, s, job, L, ctx->d_mc, ctx->d_itw);      \
        hipLaunchKernelGGL(ks1_inner_kernel<LG>, dim3(kd.M()), block, 0, s, job, kd, ctx->d_mc, ctx->d_tw,   \
                           ctx->d_itw, ctx->d_mrc);                                                           \
        hipLaunchKernelGGL(ks1_moddown_kernel<LG>, dim3(2 * L), block, 0, s, job, kd, ctx->d_mc, ctx->d_tw,  \
                           ctx->d_mrc);                                                                       \
        break;
    switch (ctx->logN) {
        LOLA_KS1_CASE(10)
        LOLA_KS1_CASE(11)
        LOLA_KS1_CASE(12)
        LOLA_KS1_CASE(13)
        LOLA_KS1_CASE(14)
        default: return set_error(LOLA_E_PARAMS, "unsupported N");
    }
#undef LOLA_KS1_CASE
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

}  // extern "C"
