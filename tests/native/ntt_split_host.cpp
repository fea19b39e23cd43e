// Host check of the NTT pass logic under every radix split the batched
// kernel is compiled with: each pass runs for every thread of the workgroup,
// then the exchange through a shared array (the device barrier), then the
// next pass, with the same pass, exchange and index functions the kernels
// call.  The forward result must equal a textbook iterative negacyclic NTT
// (itself checked against direct evaluation at odd powers of psi) at every
// index, every index must be written exactly once, and the inverse must give
// the input back.  Built with the host compiler; exit status = number of
// failed cases.
#define LOLA_HD inline
#include "../../paper_1812_10659_amd/csrc/ntt_core.hpp"

#include <array>
#include <cstdio>
#include <random>
#include <vector>

using namespace lola;
typedef unsigned __int128 u128;

static uint64_t pw(uint64_t b, uint64_t e, uint64_t m) {
    uint64_t r = 1;
    b %= m;
    while (e) {
        if (e & 1) r = (u128)r * b % m;
        b = (u128)b * b % m;
        e >>= 1;
    }
    return r;
}
static uint32_t brv(uint32_t x, int bits) {
    uint32_t r = 0;
    for (int i = 0; i < bits; i++)
        if (x >> i & 1) r |= 1u << (bits - 1 - i);
    return r;
}

using Regs = std::vector<std::array<uint32_t, NTT_E>>;
static uint32_t (&regs(Regs &X, int t))[NTT_E] { return *reinterpret_cast<uint32_t(*)[NTT_E]>(X[t].data()); }

template <int LOGN, int SPLIT, int P, bool PAD>
struct EmuFwd {
    static void run(Regs &X, uint32_t *sh, const TwPair *tw, uint32_t q) {
        constexpr int T = NttShape<LOGN, SPLIT>::T;
        using PA = FwdPassAt<LOGN, P, SPLIT>;
        for (int t = 0; t < T; t++) fwd_pass_regs<LOGN, PA::S0, PA::NS>(regs(X, t), t, tw, q);
        if constexpr (P + 1 < NttShape<LOGN, SPLIT>::NPASS) {
            using PB = FwdPassAt<LOGN, P + 1, SPLIT>;
            for (int t = 0; t < T; t++) regs_to_lds<LOGN, PA::S0, PA::NS, PAD>(regs(X, t), t, sh);
            for (int t = 0; t < T; t++) lds_to_regs<LOGN, PB::S0, PB::NS, PAD>(regs(X, t), t, sh);
            EmuFwd<LOGN, SPLIT, P + 1, PAD>::run(X, sh, tw, q);
        }
    }
};
template <int LOGN, int SPLIT, int P, bool PAD>
struct EmuInv {
    static void run(Regs &X, uint32_t *sh, const TwPair *itw, const ModConst &mc) {
        constexpr int T = NttShape<LOGN, SPLIT>::T;
        using PA = FwdPassAt<LOGN, P, SPLIT>;
        for (int t = 0; t < T; t++) inv_pass_regs<LOGN, PA::S0, PA::NS, (P == 0)>(regs(X, t), t, itw, mc);
        if constexpr (P > 0) {
            using PB = FwdPassAt<LOGN, P - 1, SPLIT>;
            for (int t = 0; t < T; t++) regs_to_lds<LOGN, PA::S0, PA::NS, PAD>(regs(X, t), t, sh);
            for (int t = 0; t < T; t++) lds_to_regs<LOGN, PB::S0, PB::NS, PAD>(regs(X, t), t, sh);
            EmuInv<LOGN, SPLIT, P - 1, PAD>::run(X, sh, itw, mc);
        }
    }
};

// Exchanges that take no workgroup barrier (both layouts keep each wave on
// its own block, pass_exchange_sync) must have every wave read back only
// residues it wrote itself.
template <int LOGN, int SPLIT, int P>
int wave_local_exchanges() {
    if constexpr (P + 1 >= NttShape<LOGN, SPLIT>::NPASS) {
        return 0;
    } else {
        using PA = FwdPassAt<LOGN, P, SPLIT>;
        using PB = FwdPassAt<LOGN, P + 1, SPLIT>;
        using A = NttPass<LOGN, PA::S0, PA::NS>;
        using B = NttPass<LOGN, PB::S0, PB::NS>;
        int bad = 0;
        if constexpr (A::WAVE_BLOCK && B::WAVE_BLOCK) {
            constexpr int N = 1 << LOGN, T = N / NTT_E;
            std::vector<int> writer(N, -1);
            for (int t = 0; t < T; t++)
                for (int r = 0; r < NTT_E; r++) writer[A::index(t, r)] = t / WAVE;
            for (int t = 0; t < T; t++)
                for (int r = 0; r < NTT_E; r++) bad += writer[B::index(t, r)] != t / WAVE;
        }
        return bad + wave_local_exchanges<LOGN, SPLIT, P + 1>();
    }
}

// The padded LDS placement: the split that regs_to_lds / lds_to_regs use
// (lds_pad(base) + lds_pad(k STR)) equals lds_pad of the register's index,
// stays inside ntt_lds_words, and is one to one.  worst[P]: the most lanes of
// one wave on one of 32 four-byte banks for one register access of pass P.
template <int LOGN, int SPLIT, int P>
int padded_placement(int (&worst)[8]) {
    if constexpr (P >= NttShape<LOGN, SPLIT>::NPASS) {
        return 0;
    } else {
        using PA = FwdPassAt<LOGN, P, SPLIT>;
        using A = NttPass<LOGN, PA::S0, PA::NS>;
        constexpr int N = 1 << LOGN, T = N / NTT_E;
        constexpr uint32_t W = ntt_lds_words<LOGN>();
        int bad = 0;
        std::vector<int> hit(W, 0);
        std::vector<uint32_t> addr((size_t)T * NTT_E);
        for (int t = 0; t < T; t++)
            for (uint32_t v = 0; v < A::PER; v++)
                for (uint32_t k = 0; k < A::SUB; k++) {
                    const uint32_t r = v * A::SUB + k;
                    const uint32_t a = lds_pad(A::base(t, v)) + lds_pad(k * A::STR);
                    bad += a != lds_pad(A::index(t, r)) || a >= W;
                    if (a < W) hit[a]++;
                    addr[(size_t)t * NTT_E + r] = a;
                }
        for (uint32_t a = 0; a < W; a++) bad += hit[a] > 1;
        int deg = 0;
        for (int w0 = 0; w0 < T; w0 += WAVE)
            for (int r = 0; r < NTT_E; r++) {
                int cnt[32] = {};
                for (int l = 0; l < WAVE && w0 + l < T; l++) {
                    const int c = ++cnt[addr[(size_t)(w0 + l) * NTT_E + r] % 32];
                    deg = c > deg ? c : deg;
                }
            }
        worst[P] = deg;
        return bad + padded_placement<LOGN, SPLIT, P + 1>(worst);
    }
}

// Forward transform of a (against ref at every index, each index written
// once), then the inverse back to a, with the plain (PAD = false) or the
// padded LDS placement.
template <int LOGN, int SPLIT, bool PAD>
int round_trip(const std::vector<uint32_t> &a, const std::vector<uint64_t> &ref, const std::vector<TwPair> &tw,
               const std::vector<TwPair> &itw, const ModConst &mc, uint32_t q) {
    constexpr int N = 1 << LOGN, T = NttShape<LOGN, SPLIT>::T;
    int bad = 0;
    Regs X(T);
    std::vector<uint32_t> sh(ntt_lds_words<LOGN>());
    for (int t = 0; t < T; t++)
        for (int k = 0; k < NTT_E; k++) X[t][k] = a[natural_index<LOGN, SPLIT>(t, k)];
    EmuFwd<LOGN, SPLIT, 0, PAD>::run(X, sh.data(), tw.data(), q);
    std::vector<int> seen(N, 0);
    for (int t = 0; t < T; t++)
        for (int k = 0; k < NTT_E; k++) {
            const uint32_t i = spectral_index<LOGN, SPLIT>(t, k);
            const uint32_t v = csub(csub(X[t][k], 2 * q), q);
            seen[i]++;
            bad += v != ref[i];
            X[t][k] = v;
        }
    for (int i = 0; i < N; i++) bad += seen[i] != 1;
    EmuInv<LOGN, SPLIT, NttShape<LOGN, SPLIT>::NPASS - 1, PAD>::run(X, sh.data(), itw.data(), mc);
    for (int t = 0; t < T; t++)
        for (int k = 0; k < NTT_E; k++) bad += csub(X[t][k], q) != a[natural_index<LOGN, SPLIT>(t, k)];
    return bad;
}

template <int LOGN, int SPLIT>
int check(uint32_t q) {
    constexpr int N = 1 << LOGN, T = NttShape<LOGN, SPLIT>::T;
    uint64_t psi = 0;
    for (uint64_t g = 2; g < q; g++)
        if (pw(g, N, q) == q - 1) {
            psi = g;
            break;
        }
    const uint64_t ipsi = pw(psi, q - 2, q);
    std::vector<TwPair> tw(N), itw(N);
    for (int k = 0; k < N; k++) {
        const uint32_t w = (uint32_t)pw(psi, brv(k, LOGN), q), iw = (uint32_t)pw(ipsi, brv(k, LOGN), q);
        tw[k] = TwPair{w, (uint32_t)(((uint64_t)w << 32) / q)};
        itw[k] = TwPair{iw, (uint32_t)(((uint64_t)iw << 32) / q)};
    }
    ModConst mc{};
    mc.q = q;
    mc.twoq = 2 * q;
    const uint64_t ninv = pw(N, q - 2, q), lw = (u128)ninv * itw[1].w % q;
    mc.ninv = (uint32_t)ninv;
    mc.ninv_shoup = (uint32_t)((ninv << 32) / q);
    mc.last_w = (uint32_t)lw;
    mc.last_w_shoup = (uint32_t)((lw << 32) / q);
    std::mt19937_64 rng(LOGN * 100000 + SPLIT);
    std::vector<uint32_t> a(N);
    for (auto &v : a) v = (uint32_t)(rng() % q);
    // textbook iterative transform (Cooley-Tukey, twiddles psi^brv(m + i))
    std::vector<uint64_t> ref(a.begin(), a.end());
    for (int m = 1, t = N; m < N; m *= 2) {
        t /= 2;
        for (int i = 0; i < m; i++)
            for (int j = 2 * i * t; j < 2 * i * t + t; j++) {
                const uint64_t U = ref[j], V = (u128)ref[j + t] * tw[m + i].w % q;
                ref[j] = (U + V) % q;
                ref[j + t] = (U + q - V) % q;
            }
    }
    int bad = 0;
    for (int k = 0; k < N; k += N / 8) {   // the textbook transform is evaluation at psi^(2 brv(k) + 1)
        const uint64_t x = pw(psi, 2 * brv(k, LOGN) + 1, q);
        uint64_t acc = 0;
        for (int j = N - 1; j >= 0; j--) acc = ((u128)acc * x + a[j]) % q;
        bad += acc != ref[k];
    }
    bad += round_trip<LOGN, SPLIT, false>(a, ref, tw, itw, mc, q) + round_trip<LOGN, SPLIT, true>(a, ref, tw, itw, mc, q);
    bad += wave_local_exchanges<LOGN, SPLIT, 0>();
    if (spectral_vec4<LOGN, SPLIT>()) {   // 16-byte accesses: registers 4r..4r+3 are 4 aligned neighbours
        for (int t = 0; t < T; t++)
            for (int r = 0; r < NTT_E; r += 4)
                for (int k = 0; k < 4; k++)
                    bad += spectral_index<LOGN, SPLIT>(t, r + k) != spectral_index<LOGN, SPLIT>(t, r) + k ||
                           spectral_index<LOGN, SPLIT>(t, r) % 4 != 0;
    }
    int worst[8] = {};
    bad += padded_placement<LOGN, SPLIT, 0>(worst);
    // at N = 16384 the exchanges of every pass but the last (which moves
    // 16-byte groups) take the minimum of two lanes per bank
    if (LOGN == 14 && (SPLIT == 0 || SPLIT == 4433))
        for (int p = 0; p + 1 < NttShape<LOGN, SPLIT>::NPASS; p++) bad += worst[p] > 2;
    std::printf("N=%d split=%d (passes %d) q=%u lanes per bank", N, SPLIT, NttShape<LOGN, SPLIT>::NPASS, q);
    for (int p = 0; p < NttShape<LOGN, SPLIT>::NPASS; p++) std::printf(" %d", worst[p]);
    std::printf(": %s\n", bad ? "FAIL" : "ok");
    return bad != 0;
}

int main() {
    const uint32_t q30 = 1073643521u, q14 = 1071513601u;   // both 1 mod 2^15
    int fails = 0;
    fails += check<10, 0>(q30) + check<10, 244>(q30) + check<10, 424>(q30) + check<10, 433>(q30) +
             check<10, 334>(q30);
    fails += check<11, 0>(q30) + check<11, 344>(q30) + check<11, 434>(q30) + check<11, 3332>(q30);
    fails += check<12, 0>(q30) + check<12, 3333>(q30) + check<12, 4332>(q30) + check<12, 2334>(q30);
    fails += check<13, 0>(q30) + check<13, 4414>(q30) + check<13, 1444>(q30) + check<13, 4432>(q30) +
             check<13, 4333>(q30) + check<13, 3334>(q30);
    fails += check<14, 0>(q14) + check<14, 4424>(q14) + check<14, 4244>(q14) + check<14, 2444>(q14) +
             check<14, 4433>(q14) + check<14, 3443>(q14) + check<14, 3344>(q14);
    return fails;
}
