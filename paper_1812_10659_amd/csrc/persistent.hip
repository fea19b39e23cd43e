// Persistent work-queue kernel for chains of rotations with uneven lengths.
//
// One launch of G workgroups.  A workgroup takes the next chain from a global
// counter (chains are ordered longest first, so the queue balances itself),
// runs all of that chain's rotations back to back -- each rotation a complete
// key switch done by the workgroup alone (digits, per-modulus transforms and
// key inner products, mod-down) with its own scratch -- and takes the next
// chain.  Workgroups never wait on each other; each leaves the loop once the
// counter has passed the number of chains, so the grid always drains.
#include "ks_core.hpp"
#include "program.hpp"

namespace lola {

struct ChainDesc {
    const uint32_t *in;     // [2][L][N] first input (not modified)
    uint32_t *out;          // [2][L][N] result of the last rotation
    uint32_t *tmp;          // [2][L][N] ping-pong buffer
    uint32_t n_steps;
    uint32_t first;         // index of the chain's first step in the step arrays
};
struct ChainStep {
    const uint32_t *key;    // switching key of the step's Galois element
    uint32_t galois;
    uint32_t pad;
};

__global__ void chain_counter_reset(uint32_t *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// One rotation by one workgroup: out = rotate(in) under key, through the
// three key-switch stages in turn (scratch: (4L+2K) N words of its own).
// KFIX = 1: contexts with one prime per digit (the shape fixed at compile
// time, which keeps the two-prime branches out of this large kernel).
template <int LOGN, int KFIX>
__device__ void wg_rotate(const uint32_t *in, uint32_t *out, const uint32_t *key, uint32_t g, const KsDims kd,
                          uint32_t *scr, uint32_t *sh, const ModConst *mcs, const TwPair *tw,
                          const TwPair *itw, const MrcConst *mrc) {
    const uint32_t L = kd.L;
    const uint32_t *c1 = in + ((size_t)L << LOGN);
    // plain LDS placement throughout, in two halves of N words (the padded
    // placement's larger buffer measured slower inside this kernel)
    for (uint32_t i = 0; i < L; ++i) ks_stage_digit<LOGN, false>(c1, g, scr, i, L, sh, mcs[i], itw, false);
    __syncthreads();
    for (uint32_t j = 0; j < kd.M(); ++j) {
        // the default radix split here: the 4433 split that suits the
        // batched inner kernel measured slower inside this larger kernel
        ks_stage_inner<LOGN, 0, (1u << LOGN), KFIX, false, true>(key, scr, j, kd, sh, mcs[j], tw, itw, mrc, c1, g);
        __syncthreads();   // the next target's transforms reuse both LDS halves
    }
    const uint32_t P = mcs[L].q;
    for (uint32_t c = 0; c < 2; ++c)
        for (uint32_t j = 0; j < L; ++j)
            ks_stage_moddown<LOGN, false, 0, KFIX>(scr, j, c, kd, c == 0 ? in : nullptr, g, nullptr, out, sh, mcs[j], tw,
                                                   mrc, P);
    __syncthreads();   // out is the next rotation's input
}

template <int LOGN, int KFIX>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void chain_persistent_kernel(
    const ChainDesc *__restrict__ chains, uint32_t n_chains, const ChainStep *__restrict__ steps,
    uint32_t *__restrict__ counter, uint32_t *__restrict__ scratch, size_t scratch_per_wg, const KsDims kd,
    const ModConst *__restrict__ mcs, const TwPair *__restrict__ tw, const TwPair *__restrict__ itw,
    const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[2 << LOGN];   // two halves of N words: plain placement only
    __shared__ uint32_t item;
    uint32_t *scr = scratch + scratch_per_wg * blockIdx.x;
    for (;;) {
        if (threadIdx.x == 0) item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t k = item;
        __syncthreads();
        if (k >= n_chains) break;   // every workgroup reaches this once the queue is empty
        const ChainDesc ch = chains[k];
        const uint32_t *src = ch.in;
        for (uint32_t r = 0; r < ch.n_steps; ++r) {
            uint32_t *dst = ((ch.n_steps - 1 - r) & 1) ? ch.tmp : ch.out;
            const ChainStep st = steps[ch.first + r];
            wg_rotate<LOGN, KFIX>(src, dst, st.key, st.galois, kd, scr, sh, mcs, tw, itw, mrc);
            src = dst;
        }
    }
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_rotate_chains(lola_ctx *ctx, const lola_chain *chains, uint32_t n, uint32_t n_wg, lola_stream stream) {
    if (!ctx || (!chains && n)) return set_error(LOLA_E_INVAL, "null argument");
    if (n == 0) return LOLA_OK;
    hipStream_t s = (hipStream_t)stream;
    // longest chains first
    std::vector<uint32_t> order(n);
    for (uint32_t k = 0; k < n; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return chains[a].n_steps > chains[b].n_steps; });
    std::vector<ChainDesc> cd;
    std::vector<ChainStep> st;
    for (uint32_t k : order) {
        const lola_chain &c = chains[k];
        if (!c.in_dev || !c.out_dev || !c.tmp_dev || (c.n_steps && (!c.galois || !c.keys)))
            return set_error(LOLA_E_INVAL, "chain buffers missing");
        if (c.out_dev == c.in_dev || c.tmp_dev == c.in_dev || c.out_dev == c.tmp_dev)
            return set_error(LOLA_E_INVAL, "chain buffers must be distinct");
        cd.push_back(ChainDesc{c.in_dev, c.out_dev, c.tmp_dev, c.n_steps, (uint32_t)st.size()});
        for (uint32_t r = 0; r < c.n_steps; ++r) {
            const uint32_t g = c.galois[r];
            if (!c.keys[r]) return set_error(LOLA_E_NOKEY, "chain step without key");
            if (g == 0 || !(g & 1) || g >= 2 * ctx->N) return set_error(LOLA_E_INVAL, "bad Galois element in chain");
            st.push_back(ChainStep{c.keys[r], g, 0});
        }
    }
    if (n_wg == 0) n_wg = 256;
    n_wg = std::min(n_wg, n);
    const size_t per = ks_scratch_words(ctx);
    void *buf = nullptr;
    int rc = scratch_get(ctx, per * n_wg * 4 + 256, &buf);
    if (rc) return rc;
    uint32_t *counter = (uint32_t *)buf;                       // first 256 bytes
    uint32_t *scr = (uint32_t *)((uint8_t *)buf + 256);
    Program p;
    const size_t oc = p.put(cd), os = p.put(st);
    void *d = nullptr;
    if ((rc = desc_upload(ctx, p.blob.data(), p.blob.size(), s, &d))) return rc;
    const ChainDesc *dcd = (const ChainDesc *)((uint8_t *)d + oc);
    const ChainStep *dst = (const ChainStep *)((uint8_t *)d + os);
    hipLaunchKernelGGL(chain_counter_reset, dim3(1), dim3(64), 0, s, counter);
    const dim3 block(ctx->N / NTT_E);
    // cost per rotation: the ciphertext in and out and the key read once; the
    // digit INTTs, the inner stage and the mod-down (those of one batched key
    // switch)
    const double rot_b = ks_whole_bytes(ctx), rot_o = ks_whole_ops(ctx);
    const uint64_t rots = st.size();
    const KsDims kd = ks_dims(ctx);
#define LOLA_CHAIN_CASE(LG)                                                                                  \
    case LG:                                                                                                 \
        if (ctx->K == 1)                                                                                     \
            LOLA_TIMED(ctx, s, KID_CHAIN, rots, rot_b * rots, rot_o * rots,                                  \
                       hipLaunchKernelGGL((chain_persistent_kernel<LG, 1>), dim3(n_wg), block, 0, s, dcd, n, dst, \
                                          counter, scr, per, kd, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc)); \
        else                                                                                                 \
            LOLA_TIMED(ctx, s, KID_CHAIN, rots, rot_b * rots, rot_o * rots,                                  \
                       hipLaunchKernelGGL((chain_persistent_kernel<LG, 0>), dim3(n_wg), block, 0, s, dcd, n, dst, \
                                          counter, scr, per, kd, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc)); \
        break;
    switch (ctx->logN) {
        LOLA_CHAIN_CASE(10)
        LOLA_CHAIN_CASE(11)
        LOLA_CHAIN_CASE(12)
        LOLA_CHAIN_CASE(13)
        LOLA_CHAIN_CASE(14)
        default: return set_error(LOLA_E_PARAMS, "unsupported N");
    }
#undef LOLA_CHAIN_CASE
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

}  // extern "C"
