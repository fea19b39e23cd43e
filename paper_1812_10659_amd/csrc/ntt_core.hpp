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
// into passes of (up to) 4; inside a pass each thread owns whole radix-16 (or
// smaller) sub-transforms and runs their butterflies in registers, so LDS is
// touched once per pass (write 16, barrier, read 16).  The forward transform
// starts in the layout of pass 0 (register k of thread t holds a[t + k T],
// coalesced in global memory) and ends in the layout of the last pass (each
// thread holds runs of 2^ns consecutive residues); the inverse goes the other
// way, so both read and write global memory in coalesced order without an
// extra staging pass.
//
// The code is __host__ __device__ so the same pass logic can be driven thread
// by thread on the CPU to check its indexing.
#pragma once
#include "modarith.hpp"

namespace lola {

constexpr int NTT_E = 16;      // residues per thread
constexpr int NTT_LOGE = 4;

template <int LOGN, int S0, int NS>
struct NttPass {
    static constexpr int N = 1 << LOGN;
    static constexpr int T = N / NTT_E;
    static constexpr int SUB = 1 << NS;          // sub-transform length
    static constexpr int PER = NTT_E / SUB;      // sub-transforms per thread
    static constexpr int STR = N >> (S0 + NS);   // stride between its residues
    // Global index held by register r = v*SUB + k of thread tid.
    LOLA_HD static int base(int tid, int v) {
        int u = tid + v * T;
        return (u / STR) * (N >> S0) + (u % STR);
    }
    LOLA_HD static int index(int tid, int r) { return base(tid, r / SUB) + (r % SUB) * STR; }
};

template <int LOGN>
struct NttShape {
    static constexpr int N = 1 << LOGN;
    static constexpr int T = N / NTT_E;
    static constexpr int NPASS = (LOGN + NTT_LOGE - 1) / NTT_LOGE;
    static constexpr int LAST_S0 = (NPASS - 1) * NTT_LOGE;
    static constexpr int LAST_NS = LOGN - LAST_S0;
    using First = NttPass<LOGN, 0, (LOGN < NTT_LOGE ? LOGN : NTT_LOGE)>;
    using Last = NttPass<LOGN, LAST_S0, LAST_NS>;
};

// ---- one forward pass on registers (layout of NttPass<LOGN,S0,NS>) ----
template <int LOGN, int S0, int NS>
LOLA_HD void fwd_pass_regs(uint32_t (&x)[NTT_E], int tid, const uint32_t *__restrict__ tw,
                           const uint32_t *__restrict__ twp, uint32_t q) {
    using PS = NttPass<LOGN, S0, NS>;
    const uint32_t twoq = 2 * q;
#pragma unroll
    for (int sg = 0; sg < NS; ++sg) {
        const int s = S0 + sg;
        const int h = PS::SUB >> (sg + 1);
#pragma unroll
        for (int v = 0; v < PS::PER; ++v) {
            const int b = PS::base(tid, v);
#pragma unroll
            for (int k = 0; k < PS::SUB; ++k) {
                if (k & h) continue;
                const int gi = (1 << s) + ((b + k * PS::STR) >> (LOGN - s));
                const uint32_t w = tw[gi], wp = twp[gi];
                uint32_t X = csub(x[v * PS::SUB + k], twoq);
                uint32_t Tm = shoup_lazy(x[v * PS::SUB + k + h], w, wp, q);
                x[v * PS::SUB + k] = X + Tm;
                x[v * PS::SUB + k + h] = X - Tm + twoq;
            }
        }
    }
}

// ---- one inverse pass on registers (stages S0+NS-1 down to S0) ----
template <int LOGN, int S0, int NS, bool LASTSTAGE_SCALE>
LOLA_HD void inv_pass_regs(uint32_t (&x)[NTT_E], int tid, const uint32_t *__restrict__ itw,
                           const uint32_t *__restrict__ itwp, const ModConst &mc) {
    using PS = NttPass<LOGN, S0, NS>;
    const uint32_t q = mc.q, twoq = mc.twoq;
#pragma unroll
    for (int sg = NS - 1; sg >= 0; --sg) {
        const int s = S0 + sg;
        const int h = PS::SUB >> (sg + 1);
#pragma unroll
        for (int v = 0; v < PS::PER; ++v) {
            const int b = PS::base(tid, v);
#pragma unroll
            for (int k = 0; k < PS::SUB; ++k) {
                if (k & h) continue;
                uint32_t U = x[v * PS::SUB + k], V = x[v * PS::SUB + k + h];
                if (LASTSTAGE_SCALE && s == 0) {
                    // N^-1 folded in: (U+V) N^-1 and (U-V) psi^-brv(1) N^-1.
                    x[v * PS::SUB + k] = shoup_lazy(U + V, mc.ninv, mc.ninv_shoup, q);
                    x[v * PS::SUB + k + h] = shoup_lazy(U - V + twoq, mc.last_w, mc.last_w_shoup, q);
                } else {
                    const int gi = (1 << s) + ((b + k * PS::STR) >> (LOGN - s));
                    x[v * PS::SUB + k] = csub(U + V, twoq);
                    x[v * PS::SUB + k + h] = shoup_lazy(U - V + twoq, itw[gi], itwp[gi], q);
                }
            }
        }
    }
}

template <int LOGN, int S0, int NS>
LOLA_HD void regs_to_lds(const uint32_t (&x)[NTT_E], int tid, uint32_t *sh) {
    using PS = NttPass<LOGN, S0, NS>;
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) sh[PS::index(tid, r)] = x[r];
}

template <int LOGN, int S0, int NS>
LOLA_HD void lds_to_regs(uint32_t (&x)[NTT_E], int tid, const uint32_t *sh) {
    using PS = NttPass<LOGN, S0, NS>;
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = sh[PS::index(tid, r)];
}

// Pass p of the forward transform covers stages [4p, min(4p+4, LOGN)).
template <int LOGN, int P>
struct FwdPassAt {
    static constexpr int S0 = P * NTT_LOGE;
    static constexpr int NS = (LOGN - S0) < NTT_LOGE ? (LOGN - S0) : NTT_LOGE;
};

#if defined(__HIP_DEVICE_COMPILE__)
#define LOLA_BARRIER() __syncthreads()
#else
#define LOLA_BARRIER() ((void)0)
#endif

// Device-side driver.  x enters in the first pass's layout and leaves in the
// last pass's layout (reduced to [0, q)).  sh: N words of LDS.  The caller
// must not touch sh between the call's start and end; a barrier is taken at
// entry so a previous use of sh by the same workgroup is complete.
template <int LOGN, int P = 0>
struct FwdDriver {
    LOLA_HD static void run(uint32_t (&x)[NTT_E], int tid, uint32_t *sh, const uint32_t *tw,
                            const uint32_t *twp, uint32_t q) {
        constexpr int NPASS = NttShape<LOGN>::NPASS;
        using PA = FwdPassAt<LOGN, P>;
        fwd_pass_regs<LOGN, PA::S0, PA::NS>(x, tid, tw, twp, q);
        if constexpr (P + 1 < NPASS) {
            using PB = FwdPassAt<LOGN, P + 1>;
            LOLA_BARRIER();
            regs_to_lds<LOGN, PA::S0, PA::NS>(x, tid, sh);
            LOLA_BARRIER();
            lds_to_regs<LOGN, PB::S0, PB::NS>(x, tid, sh);
            FwdDriver<LOGN, P + 1>::run(x, tid, sh, tw, twp, q);
        }
    }
};

template <int LOGN>
LOLA_HD void ntt_fwd_regs(uint32_t (&x)[NTT_E], int tid, uint32_t *sh, const uint32_t *tw,
                          const uint32_t *twp, uint32_t q) {
    FwdDriver<LOGN, 0>::run(x, tid, sh, tw, twp, q);
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = csub(csub(x[r], 2 * q), q);
}

// Inverse: x enters in the last forward pass's layout (values in [0, 2q))
// and leaves in the first pass's layout, reduced to [0, q).
template <int LOGN, int P>
struct InvDriver {
    LOLA_HD static void run(uint32_t (&x)[NTT_E], int tid, uint32_t *sh, const uint32_t *itw,
                            const uint32_t *itwp, const ModConst &mc) {
        using PA = FwdPassAt<LOGN, P>;
        inv_pass_regs<LOGN, PA::S0, PA::NS, (P == 0)>(x, tid, itw, itwp, mc);
        if constexpr (P > 0) {
            using PB = FwdPassAt<LOGN, P - 1>;
            LOLA_BARRIER();
            regs_to_lds<LOGN, PA::S0, PA::NS>(x, tid, sh);
            LOLA_BARRIER();
            lds_to_regs<LOGN, PB::S0, PB::NS>(x, tid, sh);
            InvDriver<LOGN, P - 1>::run(x, tid, sh, itw, itwp, mc);
        }
    }
};

template <int LOGN>
LOLA_HD void ntt_inv_regs(uint32_t (&x)[NTT_E], int tid, uint32_t *sh, const uint32_t *itw,
                          const uint32_t *itwp, const ModConst &mc) {
    InvDriver<LOGN, NttShape<LOGN>::NPASS - 1>::run(x, tid, sh, itw, itwp, mc);
#pragma unroll
    for (int r = 0; r < NTT_E; ++r) x[r] = csub(x[r], mc.q);
}

// Global index of register r in the forward input / inverse output layout.
template <int LOGN>
LOLA_HD int natural_index(int tid, int r) { return NttShape<LOGN>::First::index(tid, r); }
// Global index of register r in the forward output / inverse input layout.
template <int LOGN>
LOLA_HD int spectral_index(int tid, int r) { return NttShape<LOGN>::Last::index(tid, r); }

}  // namespace lola
