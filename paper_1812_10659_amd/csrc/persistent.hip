// Persistent work-queue kernel for chains of rotations with uneven lengths.
//
// One launch of G workgroups.  A workgroup takes the next chain from a global
// counter (chains are ordered longest first, so the queue balances itself),
// runs all of that chain's rotations back to back -- each rotation a complete
// key switch done by the workgroup alone (digits, per-modulus transforms and
// key inner products, mod-down) with its own scratch -- and takes the next
// chain.  Workgroups never wait on each other; each leaves the loop once the
// counter has passed the number of chains, so the grid always drains.
#include "ntt_core.hpp"
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

__device__ __forceinline__ uint32_t chain_perm(uint32_t idx, uint32_t g, uint32_t logN) {
    return g > 1 ? galois_src_index(idx, g, logN) : idx;
}

// One rotation by one workgroup: out = rotate(in) under key.
template <int LOGN>
__device__ void wg_rotate(const uint32_t *in, uint32_t *out, const uint32_t *key, uint32_t g, uint32_t L,
                          uint32_t *scr, uint32_t *sh, const ModConst *mcs, const TwPair *tw,
                          const TwPair *itw, const MrcConst *mrc) {
    constexpr uint32_t N = 1u << LOGN;
    const uint32_t M = L + 1;
    const uint32_t *c0 = in, *c1 = in + (size_t)L * N;
    uint32_t *D = scr, *Xp = scr + (size_t)L * N, *U = scr + (size_t)2 * L * N, *UP = scr + (size_t)4 * L * N;
    // digits: sigma_g(c1_i) kept in NTT form, inverse transform to coefficients
    for (uint32_t i = 0; i < L; ++i) {
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        uint32_t x[NTT_E];
        const uint32_t *xi = c1 + ((size_t)i << LOGN);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) {
            const uint32_t idx = spectral_index<LOGN>(tid, r);
            x[r] = xi[chain_perm(idx, g, LOGN)];
            Xp[((size_t)i << LOGN) + idx] = x[r];
        }
        uint32_t ii = i;
        asm volatile("" : "+s"(ii));
        ntt_inv_regs<LOGN>(x, tid, sh, itw + ((size_t)ii << LOGN), mcs[ii]);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) D[((size_t)i << LOGN) + natural_index<LOGN>(tid, r)] = x[r];
    }
    __syncthreads();
    // per target modulus: transforms of the digits and the key inner product
    for (uint32_t j = 0; j <= L; ++j) {
        uint32_t jj = j;
        asm volatile("" : "+s"(jj));
        const ModConst mc = mcs[jj];
        uint32_t a0[NTT_E], a1[NTT_E];
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) a0[r] = a1[r] = 0;
        for (uint32_t i = 0; i < L; ++i) {
            uint32_t tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            uint32_t x[NTT_E];
            if (i == jj) {
#pragma unroll
                for (int r = 0; r < NTT_E; ++r) x[r] = Xp[((size_t)i << LOGN) + spectral_index<LOGN>(tid, r)];
            } else {
#pragma unroll
                for (int r = 0; r < NTT_E; ++r)
                    x[r] = reduce32(D[((size_t)i << LOGN) + natural_index<LOGN>(tid, r)], mc.q, mc.one_shoup);
                uint32_t j2 = jj;
                asm volatile("" : "+s"(j2));
                ntt_fwd_regs<LOGN>(x, tid, sh, tw + ((size_t)j2 << LOGN), mc.q);
            }
            uint32_t koff = i * 2 * M + jj;
            asm volatile("" : "+s"(koff));
            const uint32_t *kb = key + ((size_t)koff << LOGN), *ka = key + ((size_t)(koff + M) << LOGN);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) {
                const uint32_t idx = spectral_index<LOGN>(tid, r);
                a0[r] = add_mod(a0[r], mont_mul(x[r], kb[idx], mc.q, mc.qneg_inv), mc.q);
                a1[r] = add_mod(a1[r], mont_mul(x[r], ka[idx], mc.q, mc.qneg_inv), mc.q);
            }
        }
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        if (jj < L) {
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) {
                const uint32_t idx = spectral_index<LOGN>(tid, r);
                U[((size_t)jj << LOGN) + idx] = a0[r];
                U[((size_t)(L + jj) << LOGN) + idx] = a1[r];
            }
        } else {
            ntt_inv_regs<LOGN>(a0, tid, sh, itw + ((size_t)jj << LOGN), mc);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) UP[natural_index<LOGN>(tid, r)] = a0[r];
            uint32_t tid2 = tid;
            asm volatile("" : "+v"(tid2));
            ntt_inv_regs<LOGN>(a1, tid2, sh, itw + ((size_t)jj << LOGN), mc);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) UP[N + natural_index<LOGN>(tid2, r)] = a1[r];
        }
    }
    __syncthreads();
    // mod-down by P and the automorphism of c0
    const uint32_t P = mcs[L].q, halfP = P >> 1;
    for (uint32_t c = 0; c < 2; ++c)
        for (uint32_t j = 0; j < L; ++j) {
            uint32_t jj = j;
            asm volatile("" : "+s"(jj));
            uint32_t tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            const ModConst mc = mcs[jj];
            uint32_t x[NTT_E];
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) {
                const uint32_t v = UP[(size_t)c * N + natural_index<LOGN>(tid, r)];
                const uint32_t vr = reduce32(v, mc.q, mc.one_shoup);
                x[r] = v > halfP ? sub_mod(vr, mrc->Pq[jj], mc.q) : vr;
            }
            ntt_fwd_regs<LOGN>(x, tid, sh, tw + ((size_t)jj << LOGN), mc.q);
            const uint32_t pinv = mrc->Pinvq[jj], pinvp = mrc->Pinvqp[jj];
            const uint32_t *Uc = U + ((size_t)(c * L + jj) << LOGN);
            const uint32_t *c0j = c0 + ((size_t)jj << LOGN);
            uint32_t *o = out + ((size_t)(c * L + jj) << LOGN);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) {
                const uint32_t idx = spectral_index<LOGN>(tid, r);
                uint32_t w = shoup(sub_mod(Uc[idx], x[r], mc.q), pinv, pinvp, mc.q);
                if (c == 0) w = add_mod(w, c0j[chain_perm(idx, g, LOGN)], mc.q);
                o[idx] = w;
            }
        }
    __syncthreads();   // out is the next rotation's input
}

template <int LOGN>
__global__ __launch_bounds__((1 << LOGN) / NTT_E) void chain_persistent_kernel(
    const ChainDesc *__restrict__ chains, uint32_t n_chains, const ChainStep *__restrict__ steps,
    uint32_t *__restrict__ counter, uint32_t *__restrict__ scratch, size_t scratch_per_wg, uint32_t L,
    const ModConst *__restrict__ mcs, const TwPair *__restrict__ tw, const TwPair *__restrict__ itw,
    const MrcConst *__restrict__ mrc) {
    __shared__ uint32_t sh[1 << LOGN];
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
            wg_rotate<LOGN>(src, dst, st.key, st.galois, L, scr, sh, mcs, tw, itw, mrc);
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
#define LOLA_CHAIN_CASE(LG)                                                                                  \
    case LG:                                                                                                 \
        hipLaunchKernelGGL(chain_persistent_kernel<LG>, dim3(n_wg), block, 0, s, dcd, n, dst, counter, scr, per, \
                           ctx->L, ctx->d_mc, ctx->d_tw, ctx->d_itw, ctx->d_mrc);                             \
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
