// The three stages of one key switch as workgroup-level device functions,
// shared by the batched launches (one stage per launch, one workgroup per
// limb-sized unit) and by the persistent kernel (one workgroup runs all
// stages of a rotation).
//
// For a polynomial x (NTT form, [L][N]) and a switching key for s' -> s with
// digits D_i = x mod q_i in [0, q_i):
//   u_m = sum_i D_i * key_i   modulo every q_j and P      (key inner product)
//   out_j = (u_j - [u_P]_P) * P^-1 mod q_j                 (mod-down by P)
// A Galois automorphism sigma_g acts on NTT-form limbs as a permutation of
// evaluation points, so a rotation folds it into the loads of x and of c0.
//
// Scratch of one key switch, (4L + 2) N words:
//   D  [L][N]   digits in coefficient form          (words 0 .. L N)
//   X' [L][N]   sigma_g(x_i) in NTT form             (L N .. 2 L N)
//   U  [2][L][N] inner products mod q_j, NTT form    (2 L N .. 4 L N)
//   UP [2][N]   inner products mod P, coefficients   (4 L N .. (4L+2) N)
//
// Key layout: [i][0 = b, 1 = a][m][N], m over q_0..q_{L-1}, P, stored times
// 2^32 mod m (Montgomery form), canonical.
//
// Every index that depends only on the thread id goes through an opaque copy
// (asm volatile with a "+v" or "+s" constraint) inside loops: otherwise the
// compiler hoists all of them, and the transforms' LDS and twiddle addresses,
// out of the loops, which does not fit in the 128 registers that a
// 1024-thread workgroup allows.
#pragma once
#include "lola_internal.hpp"
#include "ntt_core.hpp"

namespace lola {

// Workgroups go to the GPU's 8 XCDs round robin by linear id.  The batched
// stages map linear id k to (job, unit) so that all `units` workgroups of a job
// land on one XCD: every XCD gets the same mix of short and long units
// (with one unit per target modulus, the special prime's unit is half again
// as long as the others, and a plain 2-D grid of L+1 = 8 units per job would
// put all of those on one XCD).  XCD x takes the contiguous block of jobs
// [x J, x J + J), J = ceil(n / 8), in order, so the few jobs it runs at once
// are neighbours in the job list; the host sorts a launch's jobs by key, and
// neighbours that share a key (one client's requests at the same rotation)
// then read it through the same L2.
constexpr uint32_t N_XCD = 8;
struct JobUnit {
    uint32_t job, unit;
};
__host__ __device__ inline JobUnit xcd_job_unit(uint32_t k, uint32_t units, uint32_t n) {
    const uint32_t x = k % N_XCD, r = k / N_XCD, per_xcd = (n + N_XCD - 1) / N_XCD;
    return JobUnit{x * per_xcd + r / units, r % units};
}
// As xcd_job_unit, for jobs whose first `lead` units are the long ones: within
// each XCD those of all its jobs come first (in job order), then the other
// units of each job in turn.  The workgroups an XCD receives are dispatched in
// block order over its CUs, so the long units start first and the launch's
// tail holds short ones (longest first, as a list schedule wants; with each
// job's long unit ahead of only its own short ones, 13 jobs on an XCD's 32
// CUs leave a tail about 10% longer).
__host__ __device__ inline JobUnit xcd_job_unit_lead(uint32_t k, uint32_t units, uint32_t lead, uint32_t n) {
    const uint32_t x = k % N_XCD, r = k / N_XCD, per_xcd = (n + N_XCD - 1) / N_XCD;
    const uint32_t head = per_xcd * lead;
    if (r < head) return JobUnit{x * per_xcd + r / lead, r % lead};
    const uint32_t t = r - head, rest = units - lead;
    return JobUnit{x * per_xcd + t / rest, lead + t % rest};
}
// Grid size for n jobs of `units` workgroups each (ids past the last job exit).
inline uint32_t xcd_grid(uint32_t n, uint32_t units) { return (n + N_XCD - 1) / N_XCD * N_XCD * units; }

// v = the limb src (N words, NTT form) read through sigma_g at this thread's
// positions of the transform's output layout.  Without an automorphism
// (g <= 1) a plain 16-byte-per-lane read; otherwise the limb is staged in LDS
// with coalesced 16-byte loads and gathered from there (a gather straight from
// global memory touches a different cache line per lane).  g is the same for
// the whole workgroup.  Uses sh (N words) between two workgroup barriers.
template <int LOGN, int SPLIT = 0>
__device__ __forceinline__ void ks_read_sigma(const uint32_t *src, uint32_t g, uint32_t tid, uint32_t *sh,
                                              uint32_t (&v)[NTT_E]) {
    constexpr uint32_t N = 1u << LOGN, T = N / NTT_E;
    const GBuf S = gbuf(src, N);
    if (g <= 1) {
        load_spectral<LOGN, SPLIT>(S, tid, v);
        return;
    }
    __syncthreads();   // earlier readers of sh are done
#pragma unroll
    for (uint32_t r = 0; r < NTT_E / 4; ++r) {
        const uint32_t w = 4 * (tid + r * T);
        const u32x4 q = gld4(S, w);
        sh[w] = q.x, sh[w + 1] = q.y, sh[w + 2] = q.z, sh[w + 3] = q.w;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) v[r] = sh[galois_src_index(spectral_index<LOGN, SPLIT>(tid, r), g, LOGN)];
}

// Stage 1 for digit i: X'_i = sigma_g(x_i) (kept), D_i = INTT(X'_i).
// SPLIT / PAD: the transform's radix split and LDS placement (every choice
// reads and writes the same global layouts).
template <int LOGN, bool PAD = true, int SPLIT = 0>
__device__ __forceinline__ void ks_stage_digit(const uint32_t *x, uint32_t g, uint32_t *scratch, uint32_t i,
                                               uint32_t L, uint32_t *sh, const ModConst &mc,
                                               const TwPair *itw) {
    constexpr uint32_t N = 1u << LOGN;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t ii = i;
    asm volatile("" : "+s"(ii));
    uint32_t v[NTT_E];
    ks_read_sigma<LOGN, SPLIT>(x + ((size_t)ii << LOGN), g, tid, sh, v);
    store_spectral<LOGN, SPLIT>(gbuf(scratch + ((size_t)(L + ii) << LOGN), N), tid, v);
    // starts with a barrier
    ntt_inv_regs<LOGN, SPLIT, PAD>(v, tid, sh, itw + ((size_t)ii << LOGN), mc);
    const GBuf D = gbuf(scratch + ((size_t)ii << LOGN), N);
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) gst(D, natural_index<LOGN, SPLIT>(tid, r), v[r]);
}

// Stage 2 for target modulus j (q_j for j < L, P for j == L): for every
// digit, reduce it mod the target, transform it (j == i reuses X'_i), and
// accumulate its products with both key components.  The sums mod q_j go to
// U in NTT form; the sums mod P are brought back to coefficients into UP.
// sh: 2N words of LDS.  Consecutive transforms alternate between its halves,
// so each needs only the workgroup barrier inside its first exchange: when a
// transform starts writing a half, every wave has passed that barrier of the
// transform before it, and so has finished the one before that, the last
// user of the same half.  The caller must not have left reads of sh pending
// (a workgroup barrier since its last use of sh).
// Radix split of the inner stage's transforms (see NttShape).  Every stage
// reads and writes the canonical global layouts, so each may take its own:
// at N = 16384 passes of 4, 4, 3 and 3 stages measured 2% faster than the
// default 4, 4, 4, 2 for this stage, while the digit and mod-down stages were
// faster with the default.
template <int LOGN>
constexpr int ks_inner_split() { return LOGN == 14 ? 4433 : 0; }

// HALF: words between the two LDS halves (the transforms here take the plain
// placement, which needs N).
template <int LOGN, int KSI = ks_inner_split<LOGN>(), uint32_t HALF = (1u << LOGN)>
__device__ __forceinline__ void ks_stage_inner(const uint32_t *key, uint32_t *scratch, uint32_t j, uint32_t L,
                                               uint32_t *sh, const ModConst &mc, const TwPair *tw,
                                               const TwPair *itw) {
    constexpr uint32_t N = 1u << LOGN;
    const uint32_t M = L + 1;
    // 64-bit accumulators: every term is x * key with x < q (a transform's
    // output is canonical) and key < q, so at most 12 digits sum below
    // 12 q^2 < 2^64; one Montgomery reduction at the end.
    uint64_t a0[NTT_E], a1[NTT_E];
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) a0[r] = a1[r] = 0;
    uint32_t half = 0;   // LDS half of the next transform
    for (uint32_t i = 0; i < L; ++i) {
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        uint32_t x[NTT_E];
        if (i == j) {
            load_spectral<LOGN, KSI>(gbuf(scratch + ((size_t)(L + i) << LOGN), N), tid, x);
        } else {
            const GBuf D = gbuf(scratch + ((size_t)i << LOGN), N);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) x[r] = reduce32(gld(D, natural_index<LOGN, KSI>(tid, r)), mc.q, mc.one_shoup);
            uint32_t jj = j;
            asm volatile("" : "+s"(jj));
            ntt_fwd_regs<LOGN, true, KSI>(x, tid, sh + half * HALF, tw + ((size_t)jj << LOGN), mc.q);
            half ^= 1u;
        }
        // The key offset passes through an opaque copy placed after the
        // transform, so the key loads are not scheduled ahead of it.
        uint32_t koff = i * 2 * M + j;
        asm volatile("" : "+s"(koff));
        uint32_t kb[NTT_E], ka[NTT_E];
        load_spectral<LOGN, KSI>(gbuf(key + ((size_t)koff << LOGN), N), tid, kb);
        load_spectral<LOGN, KSI>(gbuf(key + ((size_t)(koff + M) << LOGN), N), tid, ka);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) {
            a0[r] += (uint64_t)x[r] * kb[r];
            a1[r] += (uint64_t)x[r] * ka[r];
        }
    }
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t u[NTT_E];
    if (j < L) {
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a0[r], (uint32_t)(a0[r] >> 32)}, mc);
        store_spectral<LOGN, KSI>(gbuf(scratch + ((size_t)(2 * L + j) << LOGN), N), tid, u);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a1[r], (uint32_t)(a1[r] >> 32)}, mc);
        store_spectral<LOGN, KSI>(gbuf(scratch + ((size_t)(3 * L + j) << LOGN), N), tid, u);
    } else {
        const GBuf UP0 = gbuf(scratch + ((size_t)(4 * L) << LOGN), N);
        const GBuf UP1 = gbuf(scratch + ((size_t)(4 * L + 1) << LOGN), N);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a0[r], (uint32_t)(a0[r] >> 32)}, mc);
        ntt_inv_regs<LOGN, KSI>(u, tid, sh, itw + ((size_t)j << LOGN), mc);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(UP0, natural_index<LOGN, KSI>(tid, r), u[r]);
        uint32_t tid2 = tid;
        asm volatile("" : "+v"(tid2));
        uint32_t jj = j;
        asm volatile("" : "+s"(jj));
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a1[r], (uint32_t)(a1[r] >> 32)}, mc);
        ntt_inv_regs<LOGN, KSI>(u, tid2, sh, itw + ((size_t)jj << LOGN), mc);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(UP1, natural_index<LOGN, KSI>(tid2, r), u[r]);
    }
}

// Latency form (launches of few jobs): stage 2 split into one workgroup per
// term, (x_i mod m_j) * key[i][c][j] for c = 0, 1, written canonical to the
// job's term area, and the L terms of each (j, c) summed afterwards.  A sum
// of Montgomery reductions is congruent to the reduction of the sum, and
// both are canonical, so the words equal those of ks_stage_inner.  Term
// area: limb 4L + 2 + 2 (j L + i) + c of the job's scratch.
__host__ __device__ constexpr size_t ks_term_limb(uint32_t L, uint32_t j, uint32_t i, uint32_t c) {
    return (size_t)(4 * L + 2) + 2 * ((size_t)j * L + i) + c;
}

// One term from the stored digits (ks_stage_digit), for launches whose terms
// take more than one round of workgroups.
template <int LOGN>
__device__ __forceinline__ void ks_stage_term(const uint32_t *key, uint32_t *scratch, uint32_t j, uint32_t i,
                                              uint32_t L, uint32_t *sh, const ModConst &mc, const TwPair *tw) {
    constexpr uint32_t N = 1u << LOGN;
    constexpr int KSI = ks_inner_split<LOGN>();
    const uint32_t M = L + 1;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t x[NTT_E];
    if (i == j) {
        load_spectral<LOGN, KSI>(gbuf(scratch + ((size_t)(L + i) << LOGN), N), tid, x);
    } else {
        const GBuf D = gbuf(scratch + ((size_t)i << LOGN), N);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = reduce32(gld(D, natural_index<LOGN, KSI>(tid, r)), mc.q, mc.one_shoup);
        ntt_fwd_regs<LOGN, false, KSI>(x, tid, sh, tw + ((size_t)j << LOGN), mc.q);
    }
    uint32_t koff = i * 2 * M + j;
    asm volatile("" : "+s"(koff));
    uint32_t kv[NTT_E], u[NTT_E];
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c) {
        load_spectral<LOGN, KSI>(gbuf(key + ((size_t)(koff + c * M) << LOGN), N), tid, kv);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) {
            const uint64_t a = (uint64_t)x[r] * kv[r];
            u[r] = acc_reduce_mont(Acc64{(uint32_t)a, (uint32_t)(a >> 32)}, mc);
        }
        store_spectral<LOGN, KSI>(gbuf(scratch + (ks_term_limb(L, j, i, c) << LOGN), N), tid, u);
    }
}

// Fold for (target m_j, component c): the sum of the L terms, stored where
// ks_stage_inner stores its result (U, or for P back in coefficients, UP).
template <int LOGN>
__device__ __forceinline__ void ks_stage_fold(uint32_t *scratch, uint32_t j, uint32_t c, uint32_t L, uint32_t *sh,
                                              const ModConst &mc, const TwPair *itw) {
    constexpr uint32_t N = 1u << LOGN;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t u[NTT_E], v[NTT_E];
    load_spectral<LOGN>(gbuf(scratch + (ks_term_limb(L, j, 0, c) << LOGN), N), tid, u);
    for (uint32_t i = 1; i < L; ++i) {
        load_spectral<LOGN>(gbuf(scratch + (ks_term_limb(L, j, i, c) << LOGN), N), tid, v);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = add_mod(u[r], v[r], mc.q);
    }
    if (j < L) {
        store_spectral<LOGN>(gbuf(scratch + ((size_t)((2 + c) * L + j) << LOGN), N), tid, u);
    } else {
        ntt_inv_regs<LOGN, 0, true>(u, tid, sh, itw + ((size_t)j << LOGN), mc);   // padded LDS placement
        const GBuf UP = gbuf(scratch + ((size_t)(4 * L + c) << LOGN), N);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(UP, natural_index<LOGN>(tid, r), u[r]);
    }
}

// The term of digit i for target m_j, computed straight from the input (the
// digit stage folded in).  sigma_g(x_i) is gathered through LDS; for i != j
// it is brought back to coefficients mod q_i (the digit D_i, which each
// target's workgroup recomputes: few jobs leave the GPU idle, so a kernel
// boundary costs more than the repeated transform), reduced mod m_j and
// transformed; then both key products, each reduced to a canonical term.
// The digits equal ks_stage_digit's, so the terms are those ks_stage_inner
// accumulates.
template <int LOGN>
__device__ __forceinline__ void ks_stage_term_direct(const uint32_t *x, uint32_t g, const uint32_t *key,
                                                     uint32_t *scratch, uint32_t j, uint32_t i, uint32_t L,
                                                     uint32_t *sh, const ModConst &mi, const ModConst &mj,
                                                     const TwPair *tw, const TwPair *itw) {
    constexpr uint32_t N = 1u << LOGN;
    constexpr int KSI = ks_inner_split<LOGN>();
    // the inverse transform (default split) leaves the registers in its first
    // pass's layout, which must be the layout the KSI forward transform takes
    static_assert(split_width(LOGN, 0, 0) == split_width(LOGN, KSI, 0), "first passes must match");
    const uint32_t M = L + 1;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t ii = i;
    asm volatile("" : "+s"(ii));
    uint32_t v[NTT_E];
    if (i == j) {
        ks_read_sigma<LOGN, KSI>(x + ((size_t)ii << LOGN), g, tid, sh, v);   // X'_i
    } else {
        ks_read_sigma<LOGN>(x + ((size_t)ii << LOGN), g, tid, sh, v);
        ntt_inv_regs<LOGN>(v, tid, sh, itw + ((size_t)ii << LOGN), mi);   // D_i; starts with a barrier
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) v[r] = reduce32(v[r], mj.q, mj.one_shoup);
        uint32_t jj = j;
        asm volatile("" : "+s"(jj));
        ntt_fwd_regs<LOGN, false, KSI>(v, tid, sh, tw + ((size_t)jj << LOGN), mj.q);
    }
    uint32_t koff = i * 2 * M + j;
    asm volatile("" : "+s"(koff));
    uint32_t kv[NTT_E], u[NTT_E];
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c) {
        load_spectral<LOGN, KSI>(gbuf(key + ((size_t)(koff + c * M) << LOGN), N), tid, kv);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) {
            const uint64_t a = (uint64_t)v[r] * kv[r];
            u[r] = acc_reduce_mont(Acc64{(uint32_t)a, (uint32_t)(a >> 32)}, mj);
        }
        store_spectral<LOGN, KSI>(gbuf(scratch + (ks_term_limb(L, j, i, c) << LOGN), N), tid, u);
    }
}

// Sum of the L terms of (target m_j, component c), canonical, in the default
// spectral layout.  Terms are loaded three limbs at a time, all three loads
// in flight together; limbs past the last repeat it and are not added.
template <int LOGN>
__device__ __forceinline__ void ks_sum_terms(const uint32_t *scratch, uint32_t j, uint32_t c, uint32_t L,
                                             uint32_t tid, uint32_t q, uint32_t (&u)[NTT_E]) {
    constexpr uint32_t N = 1u << LOGN, G = 3;
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) u[r] = 0;
    for (uint32_t i0 = 0; i0 < L; i0 += G) {
        uint32_t v[G][NTT_E];
#pragma unroll
        for (uint32_t b = 0; b < G; ++b)
            load_spectral<LOGN>(gbuf(scratch + (ks_term_limb(L, j, min(i0 + b, L - 1), c) << LOGN), N), tid, v[b]);
#pragma unroll
        for (uint32_t b = 0; b < G; ++b) {
            const uint32_t live = 0u - (uint32_t)(i0 + b < L);   // all ones for a real term
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) u[r] = add_mod(u[r], v[b][r] & live, q);
        }
    }
}

// The sum of the terms folded into the mod-down, for (target q_j, component
// c): the P terms summed and brought back to coefficients (u_P, recomputed by
// each target's workgroup), lifted into q_j and transformed; the q_j terms
// summed (U); then out as in ks_stage_moddown.  The sums equal ks_stage_inner's
// U and UP, so the words equal the batched form's.
template <int LOGN>
__device__ __forceinline__ void ks_stage_fold_moddown(const uint32_t *scratch, uint32_t j, uint32_t c, uint32_t L,
                                                      const uint32_t *add, uint32_t g, const uint32_t *addct,
                                                      uint32_t *out, uint32_t *sh, const ModConst &mj,
                                                      const ModConst &mP, const TwPair *tw, const TwPair *itw,
                                                      const MrcConst *mrc) {
    constexpr uint32_t N = 1u << LOGN;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t jj = j, LL = L;
    asm volatile("" : "+s"(jj), "+s"(LL));
    uint32_t x[NTT_E], u[NTT_E];
    ks_sum_terms<LOGN>(scratch, L, c, L, tid, mP.q, x);
    ntt_inv_regs<LOGN, 0, true>(x, tid, sh, itw + ((size_t)LL << LOGN), mP);   // u_P, coefficients
    // [u_P]_P mod q_j: v, or v - P for v > P/2 (see ks_stage_moddown)
    const uint32_t halfP = mP.q >> 1, negPq = mj.q - mrc->Pq[jj];
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = reduce32(x[r] + (x[r] > halfP ? negPq : 0u), mj.q, mj.one_shoup);
    ntt_fwd_regs<LOGN, false, 0, true>(x, tid, sh, tw + ((size_t)jj << LOGN), mj.q);
    ks_sum_terms<LOGN>(scratch, j, c, L, tid, mj.q, u);
    const uint32_t pinv = mrc->Pinvq[jj], pinvp = mrc->Pinvqp[jj];
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = csub(shoup_lazy(u[r] + mj.q - x[r], pinv, pinvp, mj.q), mj.q);
    if (add) {
        ks_read_sigma<LOGN>(add + ((size_t)jj << LOGN), g, tid, sh, u);   // after the transform's last use of sh
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = add_mod(x[r], u[r], mj.q);
    }
    if (addct) {
        load_spectral<LOGN>(gbuf(addct + ((size_t)(c * L + jj) << LOGN), N), tid, u);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = add_mod(x[r], u[r], mj.q);
    }
    store_spectral<LOGN>(gbuf(out + ((size_t)(c * L + jj) << LOGN), N), tid, x);
}

// Stage 3 for (target q_j, component c): lift [u_P]_P into q_j, transform,
// out = (U - lift) * P^-1, plus the optional addends: `add` ([L][N], read
// through sigma_g when g > 1: the rotation's c0 or the relinearisation's d0 /
// d1) and `addct` ([2][L][N], a whole ciphertext: fused rotate-and-add).
template <int LOGN, bool PAD = true, int SPLIT = 0>
__device__ __forceinline__ void ks_stage_moddown(const uint32_t *scratch, uint32_t j, uint32_t c, uint32_t L,
                                                 const uint32_t *add, uint32_t g, const uint32_t *addct,
                                                 uint32_t *out, uint32_t *sh, const ModConst &mc,
                                                 const TwPair *tw, const MrcConst *mrc, uint32_t P) {
    constexpr uint32_t N = 1u << LOGN;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t jj = j;
    asm volatile("" : "+s"(jj));
    // [u_P]_P mod q_j: v, or v - P for v > P/2, i.e. v + (q_j - P mod q_j);
    // v < P < 2^30 keeps the sum below 2^31 for one reduction.
    const uint32_t halfP = P >> 1, negPq = mc.q - mrc->Pq[jj];
    const GBuf UP = gbuf(scratch + ((size_t)(4 * L + c) << LOGN), N);
    uint32_t x[NTT_E];
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) {
        const uint32_t v = gld(UP, natural_index<LOGN, SPLIT>(tid, r));
        x[r] = reduce32(v + (v > halfP ? negPq : 0u), mc.q, mc.one_shoup);
    }
    ntt_fwd_regs<LOGN, false, SPLIT, PAD>(x, tid, sh, tw + ((size_t)jj << LOGN), mc.q);
    const uint32_t pinv = mrc->Pinvq[jj], pinvp = mrc->Pinvqp[jj];
    uint32_t u[NTT_E];
    load_spectral<LOGN, SPLIT>(gbuf(scratch + ((size_t)((2 + c) * L + jj) << LOGN), N), tid, u);
    // (U - lift) P^-1: U + q - lift < 2q feeds the lazy product directly
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = csub(shoup_lazy(u[r] + mc.q - x[r], pinv, pinvp, mc.q), mc.q);
    if (add) {
        ks_read_sigma<LOGN, SPLIT>(add + ((size_t)jj << LOGN), g, tid, sh, u);   // after the transform's last use of sh
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = add_mod(x[r], u[r], mc.q);
    }
    if (addct) {
        load_spectral<LOGN, SPLIT>(gbuf(addct + ((size_t)(c * L + jj) << LOGN), N), tid, u);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = add_mod(x[r], u[r], mc.q);
    }
    store_spectral<LOGN, SPLIT>(gbuf(out + ((size_t)(c * L + jj) << LOGN), N), tid, x);
}

// ---- hoisted rotations ---------------------------------------------------
// Rotations of one ciphertext by several Galois elements share its
// decomposition: the digits D_i = |c1|_{q_i} are taken before the
// automorphism, transformed to every other modulus once, and each rotation
// gathers them through sigma_g in the NTT domain (a permutation of the
// evaluation points), so its inner product needs no transform.  The key
// switch then acts on the digits sigma_g(D_i) (signed integer polynomials),
// which are still congruent to sigma_g(c1) mod q_i; the words differ from a
// plain rotation's.  Hoist area of a source, in limbs of N words: [0, L) the
// digits in coefficients, [L, 2L) a copy of c1 written by the digit stage
// (unused), and 2L + j L + i digit i transformed to modulus j (j <= L, i != j).
__host__ __device__ constexpr size_t ks_hoist_limb(uint32_t L, uint32_t j, uint32_t i) {
    return 2 * (size_t)L + (size_t)j * L + i;
}
__host__ __device__ constexpr size_t ks_hoist_limbs(uint32_t L) { return 2 * (size_t)L + (size_t)(L + 1) * L; }

// Digit i transformed to modulus j (j != i).
template <int LOGN>
__device__ __forceinline__ void ks_stage_modup(uint32_t *hoist, uint32_t j, uint32_t i, uint32_t *sh,
                                               const ModConst &mc, const TwPair *tw, uint32_t L) {
    constexpr uint32_t N = 1u << LOGN;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t x[NTT_E];
    const GBuf D = gbuf(hoist + ((size_t)i << LOGN), N);
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = reduce32(gld(D, natural_index<LOGN>(tid, r)), mc.q, mc.one_shoup);
    ntt_fwd_regs<LOGN>(x, tid, sh, tw + ((size_t)j << LOGN), mc.q);
    store_spectral<LOGN>(gbuf(hoist + (ks_hoist_limb(L, j, i) << LOGN), N), tid, x);
}

// Digit limb src (NTT form) read through sigma_g at this thread's positions:
// staged in LDS with coalesced 16-byte loads, then gathered.  Uses sh (N
// words) between two workgroup barriers.
template <int LOGN>
__device__ __forceinline__ void ks_hoist_gather(const uint32_t *src, uint32_t g, uint32_t tid, uint32_t *sh,
                                                uint32_t (&xv)[NTT_E]) {
    constexpr uint32_t N = 1u << LOGN, T = N / NTT_E;
    const GBuf S = gbuf(src, N);
    __syncthreads();   // the previous digit's gathers are done
#pragma unroll
    for (uint32_t r = 0; r < NTT_E / 4; ++r) {
        const uint32_t w = 4 * (tid + r * T);
        const u32x4 v = gld4(S, w);
        sh[w] = v.x, sh[w + 1] = v.y, sh[w + 2] = v.z, sh[w + 3] = v.w;
    }
    __syncthreads();
    // The gather addresses are the same for every digit; an opaque copy of g
    // keeps the compiler from holding all 16 across the caller's loop.
    uint32_t gi = g;
    asm volatile("" : "+s"(gi));
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) xv[r] = sh[galois_src_index(spectral_index<LOGN>(tid, r), gi, LOGN)];
}

// Inner product of one hoisted rotation for target modulus m_j: each digit's
// transform (c1's own limb when i == j) is read through sigma_g and
// multiplied by the key as in ks_stage_inner, whose results (U, or the
// special prime's sums back in coefficients) it writes to the same places.
// A data prime's workgroup forms both key components' sums; the special
// prime has one workgroup per component c, each with one 64-bit sum and one
// inverse transform (both sums live across two transforms do not fit the
// register file).
template <int LOGN>
__device__ __forceinline__ void ks_stage_hoisted_inner(const uint32_t *key, const uint32_t *x,
                                                       const uint32_t *hoist, uint32_t *scratch, uint32_t g,
                                                       uint32_t j, uint32_t c, uint32_t L, uint32_t *sh,
                                                       const ModConst &mc, const TwPair *itw) {
    constexpr uint32_t N = 1u << LOGN;
    const uint32_t M = L + 1;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t u[NTT_E];
    if (j < L) {
        uint64_t a0[NTT_E], a1[NTT_E];
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) a0[r] = a1[r] = 0;
#pragma unroll 1
        for (uint32_t i = 0; i < L; ++i) {
            uint32_t xv[NTT_E];
            ks_hoist_gather<LOGN>(i == j ? x + ((size_t)i << LOGN) : hoist + (ks_hoist_limb(L, j, i) << LOGN), g,
                                  tid, sh, xv);
            // one key component at a time: both at once (32 more registers
            // beside the 64 of the sums) spilled to scratch memory
            uint32_t koff = i * 2 * M + j;
            uint32_t kv[NTT_E];
            load_spectral<LOGN>(gbuf(key + ((size_t)koff << LOGN), N), tid, kv);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) a0[r] += (uint64_t)xv[r] * kv[r];
            koff += M;
            asm volatile("" : "+s"(koff));   // the second component's loads after the first products
            load_spectral<LOGN>(gbuf(key + ((size_t)koff << LOGN), N), tid, kv);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) a1[r] += (uint64_t)xv[r] * kv[r];
        }
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a0[r], (uint32_t)(a0[r] >> 32)}, mc);
        store_spectral<LOGN>(gbuf(scratch + ((size_t)(2 * L + j) << LOGN), N), tid, u);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a1[r], (uint32_t)(a1[r] >> 32)}, mc);
        store_spectral<LOGN>(gbuf(scratch + ((size_t)(3 * L + j) << LOGN), N), tid, u);
    } else {
        uint64_t a[NTT_E];
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) a[r] = 0;
#pragma unroll 1
        for (uint32_t i = 0; i < L; ++i) {
            uint32_t xv[NTT_E];
            ks_hoist_gather<LOGN>(hoist + (ks_hoist_limb(L, j, i) << LOGN), g, tid, sh, xv);
            uint32_t koff = i * 2 * M + c * M + j;
            asm volatile("" : "+s"(koff));
            uint32_t kv[NTT_E];
            load_spectral<LOGN>(gbuf(key + ((size_t)koff << LOGN), N), tid, kv);
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) a[r] += (uint64_t)xv[r] * kv[r];
        }
        // the transform below reuses sh, which other waves may still be
        // reading for the last digit's gather
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = acc_reduce_mont(Acc64{(uint32_t)a[r], (uint32_t)(a[r] >> 32)}, mc);
        ntt_inv_regs<LOGN>(u, tid, sh, itw + ((size_t)j << LOGN), mc);
        const GBuf UP = gbuf(scratch + ((size_t)(4 * L + c) << LOGN), N);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(UP, natural_index<LOGN>(tid, r), u[r]);
    }
}

}  // namespace lola
