// The three stages of one key switch as workgroup-level device functions,
// shared by the batched launches (one stage per launch, one workgroup per
// limb-sized unit) and by the persistent kernel (one workgroup runs all
// stages of a rotation).
//
// For a polynomial x (NTT form, [L][N]), K special primes p_0..p_{K-1}
// (P = their product) and a switching key for s' -> s whose digits are groups
// of K consecutive ciphertext primes (dn = ceil(L / K) of them; the last may
// hold fewer), with D_d = x mod Q_d in [0, Q_d) for the product Q_d of digit
// d's primes:
//   u_m = sum_d D_d * key_d   modulo every q_j and p_k    (key inner product)
//   out_j = (u_j - [u_P]_P) * P^-1 mod q_j                 (mod-down by P)
// K = 1 is one digit per prime.  A Galois automorphism sigma_g acts on
// NTT-form limbs as a permutation of evaluation points, so a rotation folds
// it into the loads of x and of c0.
//
// Scratch of one key switch, (4L + 2K) N words:
//   D  [L][N]    x_i in coefficient form, per prime    (words 0 .. L N)
//   X' [L][N]    sigma_g(x_i) in NTT form               (L N .. 2 L N)
//                (written for the latency form's term stage only)
//   U  [2][L][N] inner products mod q_j, NTT form       (2 L N .. 4 L N)
//   UP [2][K][N] inner products mod p_k, coefficients   (4 L N .. (4L+2K) N)
//
// Key layout: [d][0 = b, 1 = a][m][N], m over q_0..q_{L-1}, p_0..p_{K-1},
// stored times 2^32 mod m (Montgomery form), canonical.
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

// Key-switching shape of a context: L ciphertext primes, K special primes
// (context moduli L .. L+K-1), digits of K consecutive ciphertext primes.
struct KsDims {
    uint32_t L, K, dn;
    __host__ __device__ constexpr uint32_t M() const { return L + K; }
    __host__ __device__ constexpr uint32_t first(uint32_t d) const { return d * K; }
    __host__ __device__ constexpr uint32_t width(uint32_t d) const {
        return K == 1 ? 1u : (L - d * K < K ? L - d * K : K);   // d < dn
    }
    // digit d holds ciphertext prime j (whose X'_j is then the digit mod q_j)
    __host__ __device__ constexpr bool owns(uint32_t d, uint32_t j) const { return j < L && j / K == d; }
};
inline KsDims ks_dims(const lola_ctx *ctx) { return KsDims{ctx->L, ctx->K, (ctx->L + ctx->K - 1) / ctx->K}; }
// The shape with K fixed at compile time when KFIX = 1 (one prime per digit,
// one special prime), so that the two-prime branches compile away; KFIX = 0
// keeps the runtime shape.
template <int KFIX>
__host__ __device__ constexpr KsDims ks_fix(const KsDims kd) {
    return KFIX == 1 ? KsDims{kd.L, 1u, kd.L} : kd;
}

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

// Stage 1 for prime i: D_i = INTT(X'_i) with X'_i = sigma_g(x_i), and X'_i
// itself kept in the scratch when `keep` is set (for consumers that cannot
// read it through sigma_g from x: the latency form's term stage).
// SPLIT / PAD: the transform's radix split and LDS placement (every choice
// reads and writes the same global layouts).
template <int LOGN, bool PAD = true, int SPLIT = 0>
__device__ __forceinline__ void ks_stage_digit(const uint32_t *x, uint32_t g, uint32_t *scratch, uint32_t i,
                                               uint32_t L, uint32_t *sh, const ModConst &mc,
                                               const TwPair *itw, bool keep = true) {
    constexpr uint32_t N = 1u << LOGN;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t ii = i;
    asm volatile("" : "+s"(ii));
    uint32_t v[NTT_E];
    ks_read_sigma<LOGN, SPLIT>(x + ((size_t)ii << LOGN), g, tid, sh, v);
    if (keep) store_spectral<LOGN, SPLIT>(gbuf(scratch + ((size_t)(L + ii) << LOGN), N), tid, v);
    // starts with a barrier
    ntt_inv_regs<LOGN, SPLIT, PAD>(v, tid, sh, itw + ((size_t)ii << LOGN), mc);
    const GBuf D = gbuf(scratch + ((size_t)ii << LOGN), N);
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) gst(D, natural_index<LOGN, SPLIT>(tid, r), v[r]);
}

// Digit d mod m_j from two canonical limbs of its primes a, b:
// x mod q_a q_b = x_a + q_a y with y = (x_b - x_a) q_a^-1 mod q_b (Garner),
// in [0, q_a q_b), taken mod m_j.  Every modulus exceeds 2^29, so
// x_a < 2^30 < 2 q_b: x_b + 2 q_b - x_a is positive, below 3 q_b < 2^32 and
// congruent to x_b - x_a mod q_b, which the Shoup product takes as is.  The
// result x_a + (q_a y mod m_j, lazily < 2 m_j) lies in [0, 4 m_j): the range
// a forward transform takes as input (its first butterflies reduce it), so
// it is left unreduced.
LOLA_HD uint32_t ks_garner2(uint32_t xa, uint32_t xb, uint32_t qb, uint32_t iv, uint32_t ivp,
                                               uint32_t w, uint32_t wp, const ModConst &mj) {
    const uint32_t y = shoup(xb + 2 * qb - xa, iv, ivp, qb);
    return xa + shoup_lazy(y, w, wp, mj.q);
}

// This thread's coefficients (natural_index<LOGN, SPLIT>(tid, r)) of digit d
// mod m_j, from the coefficient-form limbs D ([L][N], limb i the canonical
// residue mod q_i), in [0, 4 m_j) for a forward transform.  A digit of one
// prime is its limb: reduced mod m_j with one special prime (moduli of any
// size), taken as is with two (every modulus exceeds 2^29, so a residue of
// one is below 4 m_j).
template <int LOGN, int SPLIT = 0>
__device__ __forceinline__ void ks_digit_to(const uint32_t *D, const KsDims &kd, uint32_t d, uint32_t j,
                                            const ModConst &mj, const MrcConst *mrc, uint32_t tid,
                                            uint32_t (&x)[NTT_E]) {
    constexpr uint32_t N = 1u << LOGN;
    const uint32_t a = kd.first(d);
    const GBuf Da = gbuf(D + ((size_t)a << LOGN), N);
    if (kd.width(d) == 1) {
        if (kd.K == 1) {
#pragma unroll
            for (int r = 0; r < NTT_E; ++r)
                x[r] = reduce32(gld(Da, natural_index<LOGN, SPLIT>(tid, r)), mj.q, mj.one_shoup);
        } else {
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) x[r] = gld(Da, natural_index<LOGN, SPLIT>(tid, r));
        }
        return;
    }
    const GBuf Db = gbuf(D + ((size_t)(a + 1) << LOGN), N);
    const uint32_t qb = mrc->gqb[d], iv = mrc->ginv[d], ivp = mrc->ginvp[d], w = mrc->gq[d][j], wp = mrc->gqp[d][j];
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) {
        const uint32_t idx = natural_index<LOGN, SPLIT>(tid, r);
        x[r] = ks_garner2(gld(Da, idx), gld(Db, idx), qb, iv, ivp, w, wp, mj);
    }
}

// [u]_P mod q_j for P = p_0 p_1, from u's canonical residues u0 mod p_0 and
// u1 mod p_1: V = u0 + p_0 z, z = (u1 - u0) p_0^-1 mod p_1, lies in [0, P),
// and the centred value is V - P when V > P/2, that is when z > (p_1 - 1)/2,
// or z = (p_1 - 1)/2 and u0 > (p_0 - 1)/2 (both primes odd); u1 + 2 p_1 - u0
// is positive and below 2^32 as in ks_garner2.  The result is left in
// [0, 3 q_j), for a forward transform: u0 < 2^30 < 2 q_j and the lazy product
// is below 2 q_j, so one subtraction of 2 q_j brings their sum below 2 q_j
// before q_j - (P mod q_j) is added.
LOLA_HD uint32_t ks_lift2(uint32_t u0, uint32_t u1, const MrcConst *mrc, uint32_t jj,
                                             const ModConst &mj) {
    const uint32_t p1 = mrc->sp1;
    const uint32_t z = shoup(u1 + 2 * p1 - u0, mrc->sp_inv, mrc->sp_invp, p1);
    // z > h1, or z = h1 and u0 > h0, as one comparison: 2z + [u0 > h0] > 2 h1
    const bool big = 2 * z + (u0 > mrc->sp_half0 ? 1u : 0u) > 2 * mrc->sp_half1;
    return csub(u0 + shoup_lazy(z, mrc->p0q[jj], mrc->p0qp[jj], mj.q), mj.twoq) + (big ? mj.q - mrc->Pq[jj] : 0u);
}

// Stage 2 for target modulus j (q_j for j < L, p_{j-L} for j >= L): for
// every digit, reduce it mod the target, transform it (a digit holding q_j
// reuses X'_j), and accumulate its products with both key components.  The
// sums mod q_j go to U in NTT form; the sums mod p_k are brought back to
// coefficients into UP.
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

// UP limb of (component c, special prime k).
__host__ __device__ constexpr size_t ks_up_limb(const KsDims &kd, uint32_t c, uint32_t k) {
    return 4 * (size_t)kd.L + (size_t)c * kd.K + k;
}

// HALF: words between the two LDS halves (the transforms here take the plain
// placement, which needs N).  LAZY: the digits' transforms leave their
// output in [0, 4 m_j) (no final reduction); each product is then below
// 4 m_j^2 and the sum of at most four below 16 m_j^2 < 2^64 (m_j < 2^30), so
// the caller may choose it when the shape has at most four digits.
// SIG: the digit holding q_j is read as sigma_g(x_j) from the input x (through
// an LDS half, like a transform) instead of from the copy ks_stage_digit keeps;
// the words are the same.
template <int LOGN, int KSI = ks_inner_split<LOGN>(), uint32_t HALF = (1u << LOGN), int KFIX = 0, bool LAZY = false,
          bool SIG = false>
__device__ __forceinline__ void ks_stage_inner(const uint32_t *key, uint32_t *scratch, uint32_t j, const KsDims kd_,
                                               uint32_t *sh, const ModConst &mc, const TwPair *tw,
                                               const TwPair *itw, const MrcConst *mrc,
                                               const uint32_t *xin = nullptr, uint32_t g = 0) {
    constexpr uint32_t N = 1u << LOGN;
    const KsDims kd = ks_fix<KFIX>(kd_);
    const uint32_t L = kd.L, M = kd.M();
    // 64-bit accumulators: every term is x * key with x < q (a transform's
    // output is canonical; below 4q when LAZY) and key < q, so at most 12
    // digits sum below 12 q^2 < 2^64 (at most 4 below 16 q^2 when LAZY); one
    // Montgomery reduction at the end.
    uint64_t a0[NTT_E], a1[NTT_E];
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) a0[r] = a1[r] = 0;
    uint32_t half = 0;   // LDS half of the next transform
    for (uint32_t d = 0; d < kd.dn; ++d) {
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        uint32_t x[NTT_E];
        if (kd.owns(d, j)) {
            if constexpr (SIG) {
                // with an automorphism the read stages the limb in the next
                // LDS half between two barriers; the transform after it takes
                // the other half, as after a transform
                ks_read_sigma<LOGN, KSI>(xin + ((size_t)j << LOGN), g, tid, sh + half * HALF, x);
                if (g > 1) half ^= 1u;
            } else {
                load_spectral<LOGN, KSI>(gbuf(scratch + ((size_t)(L + j) << LOGN), N), tid, x);
            }
        } else {
            ks_digit_to<LOGN, KSI>(scratch, kd, d, j, mc, mrc, tid, x);
            uint32_t jj = j;
            asm volatile("" : "+s"(jj));
            ntt_fwd_regs<LOGN, true, KSI, false, LAZY ? 2 : 0>(x, tid, sh + half * HALF, tw + ((size_t)jj << LOGN),
                                                              mc.q);
            half ^= 1u;
        }
        // The key offset passes through an opaque copy placed after the
        // transform, so the key loads are not scheduled ahead of it.
        uint32_t koff = d * 2 * M + j;
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
        const GBuf UP0 = gbuf(scratch + (ks_up_limb(kd, 0, j - L) << LOGN), N);
        const GBuf UP1 = gbuf(scratch + (ks_up_limb(kd, 1, j - L) << LOGN), N);
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
// term, (D_d mod m_j) * key[d][c][j] for c = 0, 1, written canonical to the
// job's term area, and the dn terms of each (j, c) summed afterwards.  A sum
// of Montgomery reductions is congruent to the reduction of the sum, and
// both are canonical, so the words equal those of ks_stage_inner.  Term
// area: limb 4L + 2K + 2 (j dn + d) + c of the job's scratch.
__host__ __device__ constexpr size_t ks_term_limb(const KsDims &kd, uint32_t j, uint32_t d, uint32_t c) {
    return (size_t)(4 * kd.L + 2 * kd.K) + 2 * ((size_t)j * kd.dn + d) + c;
}

// One term from the stored limbs (ks_stage_digit), for launches whose terms
// take more than one round of workgroups.
template <int LOGN>
__device__ __forceinline__ void ks_stage_term(const uint32_t *key, uint32_t *scratch, uint32_t j, uint32_t d,
                                              const KsDims kd, uint32_t *sh, const ModConst &mc, const TwPair *tw,
                                              const MrcConst *mrc) {
    constexpr uint32_t N = 1u << LOGN;
    constexpr int KSI = ks_inner_split<LOGN>();
    const uint32_t M = kd.M();
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t x[NTT_E];
    if (kd.owns(d, j)) {
        load_spectral<LOGN, KSI>(gbuf(scratch + ((size_t)(kd.L + j) << LOGN), N), tid, x);
    } else {
        ks_digit_to<LOGN, KSI>(scratch, kd, d, j, mc, mrc, tid, x);
        ntt_fwd_regs<LOGN, false, KSI>(x, tid, sh, tw + ((size_t)j << LOGN), mc.q);
    }
    uint32_t koff = d * 2 * M + j;
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
        store_spectral<LOGN, KSI>(gbuf(scratch + (ks_term_limb(kd, j, d, c) << LOGN), N), tid, u);
    }
}

// Fold for (target m_j, component c): the sum of the dn terms, stored where
// ks_stage_inner stores its result (U, or for p_k back in coefficients, UP).
template <int LOGN>
__device__ __forceinline__ void ks_stage_fold(uint32_t *scratch, uint32_t j, uint32_t c, const KsDims kd,
                                              uint32_t *sh, const ModConst &mc, const TwPair *itw) {
    constexpr uint32_t N = 1u << LOGN;
    const uint32_t L = kd.L;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t u[NTT_E], v[NTT_E];
    load_spectral<LOGN>(gbuf(scratch + (ks_term_limb(kd, j, 0, c) << LOGN), N), tid, u);
    for (uint32_t d = 1; d < kd.dn; ++d) {
        load_spectral<LOGN>(gbuf(scratch + (ks_term_limb(kd, j, d, c) << LOGN), N), tid, v);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) u[r] = add_mod(u[r], v[r], mc.q);
    }
    if (j < L) {
        store_spectral<LOGN>(gbuf(scratch + ((size_t)((2 + c) * L + j) << LOGN), N), tid, u);
    } else {
        ntt_inv_regs<LOGN, 0, true>(u, tid, sh, itw + ((size_t)j << LOGN), mc);   // padded LDS placement
        const GBuf UP = gbuf(scratch + (ks_up_limb(kd, c, j - L) << LOGN), N);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(UP, natural_index<LOGN>(tid, r), u[r]);
    }
}

// The term of digit d for target m_j, computed straight from the input (the
// digit stage folded in).  sigma_g of each of the digit's limbs is gathered
// through LDS; unless the digit holds q_j, each is brought back to
// coefficients (which each target's workgroup recomputes: few jobs leave the
// GPU idle, so a kernel boundary costs more than the repeated transforms),
// the digit is reduced mod m_j and transformed; then both key products, each
// reduced to a canonical term.  The digits equal those ks_stage_digit's limbs
// give, so the terms are those ks_stage_inner accumulates.
template <int LOGN>
__device__ __forceinline__ void ks_stage_term_direct(const uint32_t *x, uint32_t g, const uint32_t *key,
                                                     uint32_t *scratch, uint32_t j, uint32_t d, const KsDims kd,
                                                     uint32_t *sh, const ModConst *mcs, const TwPair *tw,
                                                     const TwPair *itw, const MrcConst *mrc) {
    constexpr uint32_t N = 1u << LOGN;
    constexpr int KSI = ks_inner_split<LOGN>();
    // the inverse transform (default split) leaves the registers in its first
    // pass's layout, which must be the layout the KSI forward transform takes
    static_assert(split_width(LOGN, 0, 0) == split_width(LOGN, KSI, 0), "first passes must match");
    const uint32_t M = kd.M();
    const ModConst mj = mcs[j];
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t v[NTT_E];
    if (kd.owns(d, j)) {
        uint32_t jj = j;
        asm volatile("" : "+s"(jj));
        ks_read_sigma<LOGN, KSI>(x + ((size_t)jj << LOGN), g, tid, sh, v);   // X'_j
    } else {
        uint32_t a = kd.first(d);
        asm volatile("" : "+s"(a));
        ks_read_sigma<LOGN>(x + ((size_t)a << LOGN), g, tid, sh, v);
        ntt_inv_regs<LOGN>(v, tid, sh, itw + ((size_t)a << LOGN), mcs[a]);   // x_a; starts with a barrier
        if (kd.width(d) == 1) {
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) v[r] = reduce32(v[r], mj.q, mj.one_shoup);
        } else {
            uint32_t b = a + 1;
            asm volatile("" : "+s"(b));
            uint32_t vb[NTT_E];
            ks_read_sigma<LOGN>(x + ((size_t)b << LOGN), g, tid, sh, vb);
            ntt_inv_regs<LOGN>(vb, tid, sh, itw + ((size_t)b << LOGN), mcs[b]);   // x_b
            const uint32_t qb = mrc->gqb[d], iv = mrc->ginv[d], ivp = mrc->ginvp[d];
            const uint32_t w = mrc->gq[d][j], wp = mrc->gqp[d][j];
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) v[r] = ks_garner2(v[r], vb[r], qb, iv, ivp, w, wp, mj);
        }
        uint32_t jj = j;
        asm volatile("" : "+s"(jj));
        ntt_fwd_regs<LOGN, false, KSI>(v, tid, sh, tw + ((size_t)jj << LOGN), mj.q);
    }
    uint32_t koff = d * 2 * M + j;
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
        store_spectral<LOGN, KSI>(gbuf(scratch + (ks_term_limb(kd, j, d, c) << LOGN), N), tid, u);
    }
}

// Sum of the dn terms of (target m_j, component c), canonical, in the default
// spectral layout.  Terms are loaded three limbs at a time, all three loads
// in flight together; limbs past the last repeat it and are not added.
template <int LOGN>
__device__ __forceinline__ void ks_sum_terms(const uint32_t *scratch, uint32_t j, uint32_t c, const KsDims &kd,
                                             uint32_t tid, uint32_t q, uint32_t (&u)[NTT_E]) {
    constexpr uint32_t N = 1u << LOGN, G = 3;
    const uint32_t n = kd.dn;
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) u[r] = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += G) {
        uint32_t v[G][NTT_E];
#pragma unroll
        for (uint32_t b = 0; b < G; ++b)
            load_spectral<LOGN>(gbuf(scratch + (ks_term_limb(kd, j, min(i0 + b, n - 1), c) << LOGN), N), tid, v[b]);
#pragma unroll
        for (uint32_t b = 0; b < G; ++b) {
            const uint32_t live = 0u - (uint32_t)(i0 + b < n);   // all ones for a real term
#pragma unroll
            for (int r = 0; r < NTT_E; ++r) u[r] = add_mod(u[r], v[b][r] & live, q);
        }
    }
}

// The sum of the terms folded into the mod-down, for (target q_j, component
// c): the terms of each special prime summed and brought back to
// coefficients (u mod p_k, recomputed by each target's workgroup), [u]_P
// lifted into q_j and transformed; the q_j terms summed (U); then out as in
// ks_stage_moddown.  The sums equal ks_stage_inner's U and UP, so the words
// equal the batched form's.
template <int LOGN>
__device__ __forceinline__ void ks_stage_fold_moddown(const uint32_t *scratch, uint32_t j, uint32_t c, const KsDims kd,
                                                      const uint32_t *add, uint32_t g, const uint32_t *addct,
                                                      uint32_t *out, uint32_t *sh, const ModConst *mcs,
                                                      const TwPair *tw, const TwPair *itw, const MrcConst *mrc) {
    constexpr uint32_t N = 1u << LOGN;
    const ModConst mj = mcs[j];
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t jj = j, LL = kd.L;
    asm volatile("" : "+s"(jj), "+s"(LL));
    const uint32_t L = kd.L;
    uint32_t x[NTT_E], u[NTT_E];
    const ModConst m0 = mcs[LL];
    ks_sum_terms<LOGN>(scratch, L, c, kd, tid, m0.q, x);
    ntt_inv_regs<LOGN, 0, true>(x, tid, sh, itw + ((size_t)LL << LOGN), m0);   // u mod p_0, coefficients
    if (kd.K == 1) {
        // [u_P]_P mod q_j: v, or v - P for v > P/2 (see ks_stage_moddown)
        const uint32_t halfP = m0.q >> 1, negPq = mj.q - mrc->Pq[jj];
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = reduce32(x[r] + (x[r] > halfP ? negPq : 0u), mj.q, mj.one_shoup);
    } else {
        uint32_t L1 = L + 1;
        asm volatile("" : "+s"(L1));
        const ModConst m1 = mcs[L1];
        ks_sum_terms<LOGN>(scratch, L + 1, c, kd, tid, m1.q, u);
        ntt_inv_regs<LOGN, 0, true>(u, tid, sh, itw + ((size_t)L1 << LOGN), m1);   // u mod p_1
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = ks_lift2(x[r], u[r], mrc, jj, mj);
    }
    ntt_fwd_regs<LOGN, false, 0, true>(x, tid, sh, tw + ((size_t)jj << LOGN), mj.q);
    ks_sum_terms<LOGN>(scratch, j, c, kd, tid, mj.q, u);
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
// P0: the first special prime (with one special prime, P itself).
template <int LOGN, bool PAD = true, int SPLIT = 0, int KFIX = 0>
__device__ __forceinline__ void ks_stage_moddown(const uint32_t *scratch, uint32_t j, uint32_t c, const KsDims kd_,
                                                 const uint32_t *add, uint32_t g, const uint32_t *addct,
                                                 uint32_t *out, uint32_t *sh, const ModConst &mc,
                                                 const TwPair *tw, const MrcConst *mrc, uint32_t P0) {
    constexpr uint32_t N = 1u << LOGN;
    const KsDims kd = ks_fix<KFIX>(kd_);
    const uint32_t L = kd.L;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t jj = j;
    asm volatile("" : "+s"(jj));
    const GBuf UP = gbuf(scratch + (ks_up_limb(kd, c, 0) << LOGN), N);
    uint32_t x[NTT_E];
    if (kd.K == 1) {
        // [u_P]_P mod q_j: v, or v - P for v > P/2, i.e. v + (q_j - P mod q_j);
        // v < P < 2^30 keeps the sum below 2^31 for one reduction.
        const uint32_t halfP = P0 >> 1, negPq = mc.q - mrc->Pq[jj];
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) {
            const uint32_t v = gld(UP, natural_index<LOGN, SPLIT>(tid, r));
            x[r] = reduce32(v + (v > halfP ? negPq : 0u), mc.q, mc.one_shoup);
        }
    } else {
        const GBuf UP1 = gbuf(scratch + (ks_up_limb(kd, c, 1) << LOGN), N);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) {
            const uint32_t idx = natural_index<LOGN, SPLIT>(tid, r);
            x[r] = ks_lift2(gld(UP, idx), gld(UP1, idx), mrc, jj, mc);
        }
    }
    // the transform's output left in [0, 2q): (U - lift) P^-1 takes
    // U + 2q - lift, positive and below 3q < 2^32, into the lazy product
    ntt_fwd_regs<LOGN, false, SPLIT, PAD, 1>(x, tid, sh, tw + ((size_t)jj << LOGN), mc.q);
    const uint32_t pinv = mrc->Pinvq[jj], pinvp = mrc->Pinvqp[jj];
    uint32_t u[NTT_E];
    load_spectral<LOGN, SPLIT>(gbuf(scratch + ((size_t)((2 + c) * L + jj) << LOGN), N), tid, u);
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = csub(shoup_lazy(u[r] + mc.twoq - x[r], pinv, pinvp, mc.q), mc.q);
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
// decomposition: the digits D_d = |c1|_{Q_d} are taken before the
// automorphism, transformed to every other modulus once, and each rotation
// gathers them through sigma_g in the NTT domain (a permutation of the
// evaluation points), so its inner product needs no transform.  The key
// switch then acts on the digits sigma_g(D_d) (signed integer polynomials),
// which are still congruent to sigma_g(c1) mod Q_d; the words differ from a
// plain rotation's.  Hoist area of a source, in limbs of N words: [0, L) the
// limbs of c1 in coefficients, [L, 2L) a copy of c1 written by the digit
// stage (unused), and 2L + j dn + d digit d transformed to modulus j (every
// j < L + K that digit d does not hold).
__host__ __device__ constexpr size_t ks_hoist_limb(const KsDims &kd, uint32_t j, uint32_t d) {
    return 2 * (size_t)kd.L + (size_t)j * kd.dn + d;
}
__host__ __device__ constexpr size_t ks_hoist_limbs(const KsDims &kd) {
    return 2 * (size_t)kd.L + (size_t)kd.M() * kd.dn;
}

// Digit d transformed to modulus j (a modulus the digit does not hold).
template <int LOGN>
__device__ __forceinline__ void ks_stage_modup(uint32_t *hoist, uint32_t j, uint32_t d, uint32_t *sh,
                                               const ModConst &mc, const TwPair *tw, const KsDims kd,
                                               const MrcConst *mrc) {
    constexpr uint32_t N = 1u << LOGN;
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t x[NTT_E];
    ks_digit_to<LOGN>(hoist, kd, d, j, mc, mrc, tid, x);
    ntt_fwd_regs<LOGN>(x, tid, sh, tw + ((size_t)j << LOGN), mc.q);
    store_spectral<LOGN>(gbuf(hoist + (ks_hoist_limb(kd, j, d) << LOGN), N), tid, x);
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
// transform (c1's own limb when the digit holds q_j) is read through sigma_g
// and multiplied by the key as in ks_stage_inner, whose results (U, or the
// special primes' sums back in coefficients) it writes to the same places.
// A ciphertext prime's workgroup forms both key components' sums; a special
// prime has one workgroup per component c, each with one 64-bit sum and one
// inverse transform (both sums live across two transforms do not fit the
// register file).
template <int LOGN>
__device__ __forceinline__ void ks_stage_hoisted_inner(const uint32_t *key, const uint32_t *x,
                                                       const uint32_t *hoist, uint32_t *scratch, uint32_t g,
                                                       uint32_t j, uint32_t c, const KsDims kd, uint32_t *sh,
                                                       const ModConst &mc, const TwPair *itw) {
    constexpr uint32_t N = 1u << LOGN;
    const uint32_t L = kd.L, M = kd.M();
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    uint32_t u[NTT_E];
    if (j < L) {
        uint64_t a0[NTT_E], a1[NTT_E];
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) a0[r] = a1[r] = 0;
#pragma unroll 1
        for (uint32_t d = 0; d < kd.dn; ++d) {
            uint32_t xv[NTT_E];
            ks_hoist_gather<LOGN>(kd.owns(d, j) ? x + ((size_t)j << LOGN) : hoist + (ks_hoist_limb(kd, j, d) << LOGN),
                                  g, tid, sh, xv);
            // one key component at a time: both at once (32 more registers
            // beside the 64 of the sums) spilled to scratch memory
            uint32_t koff = d * 2 * M + j;
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
        for (uint32_t d = 0; d < kd.dn; ++d) {
            uint32_t xv[NTT_E];
            ks_hoist_gather<LOGN>(hoist + (ks_hoist_limb(kd, j, d) << LOGN), g, tid, sh, xv);
            uint32_t koff = d * 2 * M + c * M + j;
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
        const GBuf UP = gbuf(scratch + (ks_up_limb(kd, c, j - L) << LOGN), N);
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(UP, natural_index<LOGN>(tid, r), u[r]);
    }
}

}  // namespace lola
