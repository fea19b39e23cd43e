// Negacyclic NTT of one limb (N residues mod q) by one workgroup, held in
// registers with exchanges through LDS.
//
// Transform: a_hat[k] = a(psi^(2 brv(k) + 1)), k < N, psi a primitive 2N-th
// root mod q and brv the log2(N)-bit reversal.  Forward: Cooley-Tukey
// butterflies over stages s = 0..log2N-1 with twiddles psi^brv(2^s + i) (the
// twisted form that needs no separate pre/post multiplication); inverse:
// Gentleman-Sande butterflies with psi^-brv(2^s + i), stages in reverse, and
// N^-1 folded into the last stage.  Harvey's lazy reduction keeps forward
// values in [0, 4q) and inverse values in [0, 2q) between stages.
//
// Work split: T = N/16 threads, 16 residues per thread.  Stages are grouped
// into passes of (up to) 4 (the radix split, a template choice: see
// NttShape); inside a pass each thread owns whole radix-16 (or
// smaller) sub-transforms and runs their butterflies in registers, so LDS is
// touched once per pass (write 16, barrier, read 16).  The forward transform
// starts in the layout of pass 0 (register k of thread t holds a[t + k T],
// coalesced in global memory) and ends in the layout of the last pass (each
// thread holds runs of 2^ns consecutive residues); the inverse goes the other
// way, so both read and write global memory in coalesced order without an
// extra staging pass.
//
// Twiddles are stored as (w, floor(w 2^32 / q)) pairs and read with one 64-bit
// load.  When a pass's sub-transform stride is at least the wavefront width,
// all 64 lanes of a wave sit in the same butterfly group, so the twiddle index
// is wave-uniform; it is then moved to a scalar register and the load becomes
// a scalar load (passes 0 and, for N = 16384, 1).
//
// The code is __host__ __device__ so the same pass logic can be driven thread
// by thread on the CPU to check its indexing.
#pragma once
#include "modarith.hpp"

namespace lola {

constexpr int NTT_E = 16;      // residues per thread
constexpr int NTT_LOGE = 4;
constexpr int WAVE = 64;

template <int LOGN, int S0, int NS>
struct NttPass {
    static constexpr uint32_t N = 1u << LOGN;
    static constexpr uint32_t T = N / NTT_E;
    static constexpr uint32_t SUB = 1u << NS;          // sub-transform length
    static constexpr uint32_t PER = NTT_E / SUB;       // sub-transforms per thread
    static constexpr uint32_t STR = N >> (S0 + NS);    // stride between its residues
    // Global index held by register r = v*SUB + k of thread tid.  The wave
    // owning lanes [64w, 64w+64) takes sub-transforms [64w PER, 64(w+1) PER),
    // lane l taking l, l + 64, ... (u = 64 w PER + l + 64 v): when
    // 64*PER >= STR a wave's lanes hold one contiguous block of 64*16
    // residues, and for a fixed register neighbouring lanes touch
    // neighbouring addresses (coalesced global access).
    LOLA_HD static uint32_t base(uint32_t tid, uint32_t v) {
        const uint32_t u = (tid & ~(uint32_t)(WAVE - 1)) * PER + (tid & (uint32_t)(WAVE - 1)) + (uint32_t)WAVE * v;
        return (u / STR) * (N >> S0) + (u % STR);
    }
    static constexpr bool WAVE_BLOCK = (uint32_t)WAVE * PER >= STR;
    LOLA_HD static uint32_t index(uint32_t tid, uint32_t r) { return base(tid, r / SUB) + (r % SUB) * STR; }
};

// Radix split: how the log2(N) stages group into passes.  SPLIT = 0 takes
// passes of 4 stages from the first, the remainder last (4442 at N = 16384);
// otherwise SPLIT lists the stages of each pass as decimal digits, first pass
// first (e.g. 2444 or 4433), each between 1 and 4 and summing to log2(N).
constexpr int split_npass(int logn, int split) {
    if (split == 0) return (logn + NTT_LOGE - 1) / NTT_LOGE;
    int n = 0;
    for (int v = split; v > 0; v /= 10) ++n;
    return n;
}
// Stages of pass p (0 = first).
constexpr int split_width(int logn, int split, int p) {
    if (split == 0) return (logn - p * NTT_LOGE) < NTT_LOGE ? (logn - p * NTT_LOGE) : NTT_LOGE;
    int v = split;
    for (int k = split_npass(logn, split) - 1; k > p; --k) v /= 10;
    return v % 10;
}
// First stage of pass p.
constexpr int split_s0(int logn, int split, int p) {
    int s = 0;
    for (int k = 0; k < p; ++k) s += split_width(logn, split, k);
    return s;
}
constexpr bool split_valid(int logn, int split) {
    if (split < 0) return false;
    int total = 0;
    for (int p = 0; p < split_npass(logn, split); ++p) {
        const int w = split_width(logn, split, p);
        if (w < 1 || w > NTT_LOGE) return false;
        total += w;
    }
    return total == logn;
}

template <int LOGN, int SPLIT = 0>
struct NttShape {
    static_assert(split_valid(LOGN, SPLIT), "radix split must list passes of 1..4 stages summing to log2(N)");
    static constexpr int N = 1 << LOGN;
    static constexpr int T = N / NTT_E;
    static constexpr int NPASS = split_npass(LOGN, SPLIT);
    static constexpr int LAST_S0 = split_s0(LOGN, SPLIT, NPASS - 1);
    static constexpr int LAST_NS = LOGN - LAST_S0;
    using First = NttPass<LOGN, 0, split_width(LOGN, SPLIT, 0)>;
    using Last = NttPass<LOGN, LAST_S0, LAST_NS>;
};

// Twiddle-pair index of stage s for the butterfly group containing global
// index g: 2^s + (g >> (log2N - s)); made scalar when wave-uniform.
template <int LOGN, int S0, int NS>
LOLA_HD uint32_t tw_index(uint32_t b, uint32_t k, int s) {
    using PS = NttPass<LOGN, S0, NS>;
    uint32_t gi = (1u << s) + ((b + k * PS::STR) >> (LOGN - s));
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (PS::STR >= (uint32_t)WAVE) gi = __builtin_amdgcn_readfirstlane(gi);
#endif
    return gi;
}

// ---- one forward pass on registers (layout of NttPass<LOGN,S0,NS>) ----
template <int LOGN, int S0, int NS>
LOLA_HD void fwd_pass_regs(uint32_t (&x)[NTT_E], uint32_t tid, const TwPair *__restrict__ tw, uint32_t q) {
    using PS = NttPass<LOGN, S0, NS>;
    const uint32_t twoq = 2 * q;
#pragma unroll
    for (int sg = 0; sg < NS; ++sg) {
        const int s = S0 + sg;
        const uint32_t h = PS::SUB >> (sg + 1);
#pragma unroll
        for (uint32_t v = 0; v < PS::PER; ++v) {
            const uint32_t b = PS::base(tid, v);
#pragma unroll
            for (uint32_t k = 0; k < PS::SUB; ++k) {
                if (k & h) continue;
                const TwPair t = tw[tw_index<LOGN, S0, NS>(b, k, s)];
                const uint32_t X = csub(x[v * PS::SUB + k], twoq);
                // nT = -(w y mod q, lazily in [0, 2q)) modulo 2^32; written
                // negated so the second output is one three-input add.
                const uint32_t y = x[v * PS::SUB + k + h];
                const uint32_t nT = mulhi32(y, t.wp) * q - y * t.w;
                x[v * PS::SUB + k] = X - nT;
                x[v * PS::SUB + k + h] = X + twoq + nT;
            }
        }
    }
}

// ---- one inverse pass on registers (stages S0+NS-1 down to S0) ----
template <int LOGN, int S0, int NS, bool LASTSTAGE_SCALE>
LOLA_HD void inv_pass_regs(uint32_t (&x)[NTT_E], uint32_t tid, const TwPair *__restrict__ itw,
                           const ModConst &mc) {
    using PS = NttPass<LOGN, S0, NS>;
    const uint32_t q = mc.q, twoq = mc.twoq;
#pragma unroll
    for (int sg = NS - 1; sg >= 0; --sg) {
        const int s = S0 + sg;
        const uint32_t h = PS::SUB >> (sg + 1);
#pragma unroll
        for (uint32_t v = 0; v < PS::PER; ++v) {
            const uint32_t b = PS::base(tid, v);
#pragma unroll
            for (uint32_t k = 0; k < PS::SUB; ++k) {
                if (k & h) continue;
                uint32_t U = x[v * PS::SUB + k], V = x[v * PS::SUB + k + h];
                if (LASTSTAGE_SCALE && s == 0) {
                    // N^-1 folded in: (U+V) N^-1 and (U-V) psi^-brv(1) N^-1.
                    x[v * PS::SUB + k] = shoup_lazy(U + V, mc.ninv, mc.ninv_shoup, q);
                    x[v * PS::SUB + k + h] = shoup_lazy(U - V + twoq, mc.last_w, mc.last_w_shoup, q);
                } else {
                    const TwPair t = itw[tw_index<LOGN, S0, NS>(b, k, s)];
                    x[v * PS::SUB + k] = csub(U + V, twoq);
                    x[v * PS::SUB + k + h] = shoup_lazy(U - V + twoq, t.w, t.wp, q);
                }
            }
        }
    }
}

// LDS placement of a transform's residues, chosen per call site (PAD):
// either plain (g) or with NTT_LDS_PAD words of padding after every 64
// (g -> g + 4 floor(g / 64)).  In the middle passes a wave's lanes touch
// residues 64 or more apart for one register (e.g. stride 4 within groups of
// 4 lanes); plain, these fall on a few banks, padded they spread over all of
// them, at the price of the 256-byte strides that let pairs of accesses
// share one instruction.  Which one is faster depends on the kernel around
// the transform (measured), so both exist.  Padding by whole 16-byte groups
// keeps the 4-aligned runs of the last pass aligned.  A buffer for the
// padded placement holds N + N/16 words, one for the plain placement N
// (kept at N where only the plain one is used: the larger allocation
// measured slower in kernels that hold two buffers).
constexpr uint32_t NTT_LDS_PAD = 4;
LOLA_HD constexpr uint32_t lds_pad(uint32_t g) { return g + NTT_LDS_PAD * (g >> 6); }
template <int LOGN, bool PAD = true>
constexpr uint32_t ntt_lds_words() { return PAD ? lds_pad(1u << LOGN) : (1u << LOGN); }

// A register's index is base(tid, v) + k STR with the sub-transform's span
// STR * SUB a power of two and base mod span = u mod STR < STR, so adding
// k STR never carries out of the low 6 bits of base past what k STR itself
// carries: lds_pad(base + k STR) = lds_pad(base) + lds_pad(k STR), and the
// per-register part is a compile-time offset.
template <bool PAD>
LOLA_HD constexpr uint32_t lds_place(uint32_t g) { return PAD ? lds_pad(g) : g; }

template <int LOGN, int S0, int NS, bool PAD = false>
LOLA_HD void regs_to_lds(const uint32_t (&x)[NTT_E], uint32_t tid, uint32_t *sh) {
    using PS = NttPass<LOGN, S0, NS>;
#pragma unroll
    for (uint32_t v = 0; v < PS::PER; ++v) {
        const uint32_t pb = lds_place<PAD>(PS::base(tid, v));
#pragma unroll
        for (uint32_t k = 0; k < PS::SUB; ++k) sh[pb + lds_place<PAD>(k * PS::STR)] = x[v * PS::SUB + k];
    }
}

template <int LOGN, int S0, int NS, bool PAD = false>
LOLA_HD void lds_to_regs(uint32_t (&x)[NTT_E], uint32_t tid, const uint32_t *sh) {
    using PS = NttPass<LOGN, S0, NS>;
#pragma unroll
    for (uint32_t v = 0; v < PS::PER; ++v) {
        const uint32_t pb = lds_place<PAD>(PS::base(tid, v));
#pragma unroll
        for (uint32_t k = 0; k < PS::SUB; ++k) x[v * PS::SUB + k] = sh[pb + lds_place<PAD>(k * PS::STR)];
    }
}

// Pass P of the forward transform under radix split SPLIT.
template <int LOGN, int P, int SPLIT = 0>
struct FwdPassAt {
    static constexpr int S0 = split_s0(LOGN, SPLIT, P);
    static constexpr int NS = split_width(LOGN, SPLIT, P);
};

#if defined(__HIP_DEVICE_COMPILE__)
#define LOLA_BARRIER() __syncthreads()
// Ordering of LDS traffic among the lanes of one wave: the LDS unit serves a
// wave's instructions in order; this keeps the compiler from moving LDS
// accesses across the point (no s_barrier is issued).
#define LOLA_WAVE_SYNC()                                       \
    do {                                                       \
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
        __builtin_amdgcn_wave_barrier();                       \
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront"); \
    } while (0)
#else
#define LOLA_BARRIER() ((void)0)
#define LOLA_WAVE_SYNC() ((void)0)
#endif

// Exchange between two passes: a workgroup barrier unless every wave reads
// back exactly the block of residues it wrote.
template <int LOGN, class PA, class PB>
LOLA_HD void pass_exchange_sync() {
    if constexpr (NttPass<LOGN, PA::S0, PA::NS>::WAVE_BLOCK && NttPass<LOGN, PB::S0, PB::NS>::WAVE_BLOCK)
        LOLA_WAVE_SYNC();
    else
        LOLA_BARRIER();
}

// Device-side driver.  x enters in the first pass's layout and leaves in the
// last pass's layout (reduced to [0, q)).  sh: ntt_lds_words<LOGN, PAD>() words of LDS.  A barrier is
// taken before the first LDS write, so a previous use of sh by the same
// workgroup is complete.
// FRESH: no wave of the workgroup can still be reading sh from an earlier
// use (e.g. the caller alternates two buffers and the transform before the
// previous one ended behind a workgroup barrier), so the first exchange
// needs no barrier before its writes.
template <int LOGN, int P = 0, bool FRESH = false, int SPLIT = 0, bool PAD = false>
struct FwdDriver {
    LOLA_HD static void run(uint32_t (&x)[NTT_E], uint32_t tid, uint32_t *sh, const TwPair *tw, uint32_t q) {
        constexpr int NPASS = NttShape<LOGN, SPLIT>::NPASS;
        using PA = FwdPassAt<LOGN, P, SPLIT>;
        fwd_pass_regs<LOGN, PA::S0, PA::NS>(x, tid, tw, q);
        if constexpr (P + 1 < NPASS) {
            using PB = FwdPassAt<LOGN, P + 1, SPLIT>;
            // The first exchange of a transform waits for every earlier LDS
            // reader of the workgroup; later ones only for this wave when
            // both layouts keep each wave on its own block.
            if constexpr (P == 0) {
                if constexpr (!FRESH) LOLA_BARRIER();
            } else {
                pass_exchange_sync<LOGN, PA, PB>();
            }
            regs_to_lds<LOGN, PA::S0, PA::NS, PAD>(x, tid, sh);
            pass_exchange_sync<LOGN, PA, PB>();
            lds_to_regs<LOGN, PB::S0, PB::NS, PAD>(x, tid, sh);
            FwdDriver<LOGN, P + 1, FRESH, SPLIT, PAD>::run(x, tid, sh, tw, q);
        }
    }
};

// LAZY: how far the output is reduced, for a caller that reduces it later:
// 0 to [0, q), 1 to [0, 2q), 2 not at all ([0, 4q), the butterflies' range).
template <int LOGN, bool FRESH = false, int SPLIT = 0, bool PAD = false, int LAZY = 0>
LOLA_HD void ntt_fwd_regs(uint32_t (&x)[NTT_E], uint32_t tid, uint32_t *sh, const TwPair *tw, uint32_t q) {
    FwdDriver<LOGN, 0, FRESH, SPLIT, PAD>::run(x, tid, sh, tw, q);
    if constexpr (LAZY == 0) {
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = csub(csub(x[r], 2 * q), q);
    } else if constexpr (LAZY == 1) {
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) x[r] = csub(x[r], 2 * q);
    }
}

// Inverse: x enters in the last forward pass's layout (values in [0, 2q))
// and leaves in the first pass's layout, reduced to [0, q).
template <int LOGN, int P, int SPLIT = 0, bool PAD = false>
struct InvDriver {
    LOLA_HD static void run(uint32_t (&x)[NTT_E], uint32_t tid, uint32_t *sh, const TwPair *itw,
                            const ModConst &mc) {
        using PA = FwdPassAt<LOGN, P, SPLIT>;
        inv_pass_regs<LOGN, PA::S0, PA::NS, (P == 0)>(x, tid, itw, mc);
        if constexpr (P > 0) {
            using PB = FwdPassAt<LOGN, P - 1, SPLIT>;
            if constexpr (P == NttShape<LOGN, SPLIT>::NPASS - 1) LOLA_BARRIER();
            else pass_exchange_sync<LOGN, PA, PB>();
            regs_to_lds<LOGN, PA::S0, PA::NS, PAD>(x, tid, sh);
            pass_exchange_sync<LOGN, PA, PB>();
            lds_to_regs<LOGN, PB::S0, PB::NS, PAD>(x, tid, sh);
            InvDriver<LOGN, P - 1, SPLIT, PAD>::run(x, tid, sh, itw, mc);
        }
    }
};

template <int LOGN, int SPLIT = 0, bool PAD = false>
LOLA_HD void ntt_inv_regs(uint32_t (&x)[NTT_E], uint32_t tid, uint32_t *sh, const TwPair *itw,
                          const ModConst &mc) {
    InvDriver<LOGN, NttShape<LOGN, SPLIT>::NPASS - 1, SPLIT, PAD>::run(x, tid, sh, itw, mc);
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = csub(x[r], mc.q);
}

// Global index of register r in the forward input / inverse output layout.
template <int LOGN, int SPLIT = 0>
LOLA_HD uint32_t natural_index(uint32_t tid, uint32_t r) { return NttShape<LOGN, SPLIT>::First::index(tid, r); }
// Global index of register r in the forward output / inverse input layout.
template <int LOGN, int SPLIT = 0>
LOLA_HD uint32_t spectral_index(uint32_t tid, uint32_t r) { return NttShape<LOGN, SPLIT>::Last::index(tid, r); }

// Registers r..r+3 of the forward output layout hold four consecutive,
// 4-aligned residues when the last pass's sub-transforms have at least four
// elements (stride 1, base a multiple of the length): then they move with one
// 16-byte access per lane and neighbouring lanes touch neighbouring 16 bytes.
template <int LOGN, int SPLIT = 0>
constexpr bool spectral_vec4() {
    return NttShape<LOGN, SPLIT>::Last::SUB >= 4 && NttShape<LOGN, SPLIT>::Last::STR == 1;
}

template <int LOGN, int SPLIT = 0>
LOLA_HD void load_spectral(GBuf b, uint32_t tid, uint32_t (&y)[NTT_E]) {
    if constexpr (spectral_vec4<LOGN, SPLIT>()) {
#pragma unroll
        for (int r = 0; r < NTT_E; r += 4) {
            const u32x4 v = gld4(b, spectral_index<LOGN, SPLIT>(tid, r));
            y[r] = v.x, y[r + 1] = v.y, y[r + 2] = v.z, y[r + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) y[r] = gld(b, spectral_index<LOGN, SPLIT>(tid, r));
    }
}

template <int LOGN, int SPLIT = 0>
LOLA_HD void store_spectral(GBuf b, uint32_t tid, const uint32_t (&y)[NTT_E]) {
    if constexpr (spectral_vec4<LOGN, SPLIT>()) {
#pragma unroll
        for (int r = 0; r < NTT_E; r += 4) {
            u32x4 v;
            v.x = y[r], v.y = y[r + 1], v.z = y[r + 2], v.w = y[r + 3];
            gst4(b, spectral_index<LOGN, SPLIT>(tid, r), v);
        }
    } else {
#pragma unroll
        for (int r = 0; r < NTT_E; ++r) gst(b, spectral_index<LOGN, SPLIT>(tid, r), y[r]);
    }
}

}  // namespace lola
