// Host check of the two-prime conversions of key switching with digits of
// two primes: ks_garner2 (a digit x mod q_a q_b, from its two residues, mod
// another modulus m, left in [0, 4m)) and ks_lift2 (the centred [u]_P mod
// q_j for P = p_0 p_1, left in [0, 3 q_j)), each against the exact value from
// 128-bit integers and within its stated range, on random residues and on the
// edge residues (0, 1, q-1, and the centring threshold).  Exit status =
// number of failures.
#include "../../paper_1812_10659_amd/csrc/ks_core.hpp"

#include <cstdio>
#include <random>

using namespace lola;
typedef unsigned __int128 u128;
typedef __int128 i128;

static uint64_t pw(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1;
    a %= m;
    while (e) {
        if (e & 1) r = (uint64_t)((u128)r * a % m);
        a = (uint64_t)((u128)a * a % m);
        e >>= 1;
    }
    return r;
}
static uint64_t inv(uint64_t a, uint64_t m) { return pw(a, m - 2, m); }   // m prime
static ModConst mconst(uint32_t q) {
    ModConst c{};
    c.q = q;
    c.twoq = 2 * q;
    c.one_shoup = (uint32_t)((1ull << 32) / q);
    return c;
}

int main() {
    // ciphertext and special primes = 1 mod 2^15, all above 2^29
    const uint32_t P[] = {1073643521, 1073479681, 1073184769, 1073053697, 1072857089, 1072496641,
                          1071513601, 1071415297, 1071087617, 1070727169, 1070432257, 1069219841,
                          536903681 /* just above 2^29 */};
    const int NP = sizeof P / sizeof P[0];
    std::mt19937_64 rng(12345);
    int bad = 0;
    long checked = 0;
    for (int a = 0; a < NP; ++a)
        for (int b = 0; b < NP; ++b)
            for (int j = 0; j < NP; ++j) {
                if (a == b || j == a || j == b) continue;
                const uint64_t qa = P[a], qb = P[b], mj = P[j];
                const uint32_t iv = (uint32_t)inv(qa % qb, qb), ivp = shoup_companion(iv, (uint32_t)qb);
                const uint32_t w = (uint32_t)(qa % mj), wp = shoup_companion(w, (uint32_t)mj);
                const ModConst mc = mconst((uint32_t)mj);
                const uint32_t edge_a[] = {0, 1, (uint32_t)qa - 1, (uint32_t)(qa / 2)};
                const uint32_t edge_b[] = {0, 1, (uint32_t)qb - 1, (uint32_t)(qb / 2)};
                for (int t = 0; t < 64; ++t) {
                    const uint32_t xa = t < 16 ? edge_a[t % 4] : (uint32_t)(rng() % qa);
                    const uint32_t xb = t < 16 ? edge_b[t / 4] : (uint32_t)(rng() % qb);
                    // the integer in [0, qa qb) with these residues
                    const u128 Q = (u128)qa * qb;
                    u128 v = 0;
                    v += (u128)xa * qb % Q * inv(qb % qa, qa) % Q;
                    v += (u128)xb * qa % Q * inv(qa % qb, qb) % Q;
                    v %= Q;
                    const uint32_t want = (uint32_t)(v % mj);
                    const uint32_t got = ks_garner2(xa, xb, (uint32_t)qb, iv, ivp, w, wp, mc);
                    ++checked;
                    if (got >= 4 * mj || got % mj != want) {
                        if (bad < 5) printf("garner2 qa=%llu qb=%llu m=%llu xa=%u xb=%u got %u want %u\n",
                                            (unsigned long long)qa, (unsigned long long)qb, (unsigned long long)mj,
                                            xa, xb, got, want);
                        ++bad;
                    }
                }
                // lift: p_0 = P[a], p_1 = P[b], target q_j
                MrcConst m{};
                m.sp1 = (uint32_t)qb;
                m.sp_inv = iv;
                m.sp_invp = ivp;
                m.sp_half0 = (uint32_t)((qa - 1) / 2);
                m.sp_half1 = (uint32_t)((qb - 1) / 2);
                m.p0q[0] = w;
                m.p0qp[0] = wp;
                const uint64_t Pm = (uint64_t)((u128)qa * qb % mj);
                m.Pq[0] = (uint32_t)Pm;
                const u128 PP = (u128)qa * qb;
                // u0, u1 residues of: random values, and values around P/2
                for (int t = 0; t < 64; ++t) {
                    u128 V;
                    if (t < 8) V = PP / 2 - 4 + t;   // P/2 - 4 .. P/2 + 3
                    else if (t < 12) V = (u128)(t - 8);
                    else if (t < 16) V = PP - 1 - (t - 12);
                    else V = (((u128)rng() << 64) | rng()) % PP;
                    const uint32_t u0 = (uint32_t)(V % qa), u1 = (uint32_t)(V % qb);
                    const i128 c = V > PP / 2 ? (i128)V - (i128)PP : (i128)V;   // centred
                    i128 r = c % (i128)mj;
                    if (r < 0) r += mj;
                    const uint32_t got = ks_lift2(u0, u1, &m, 0, mc);
                    ++checked;
                    if (got >= 3 * mj || got % mj != (uint32_t)r) {
                        if (bad < 5) printf("lift2 p0=%llu p1=%llu q=%llu got %u want %u\n", (unsigned long long)qa,
                                            (unsigned long long)qb, (unsigned long long)mj, got, (uint32_t)r);
                        ++bad;
                    }
                }
            }
    // digit shapes: widths and ownership
    for (uint32_t L = 1; L <= 12; ++L)
        for (uint32_t K = 1; K <= 2; ++K) {
            const KsDims kd{L, K, (L + K - 1) / K};
            uint32_t covered = 0;
            for (uint32_t d = 0; d < kd.dn; ++d) {
                covered += kd.width(d);
                if (kd.width(d) < 1 || kd.width(d) > K) ++bad;
                for (uint32_t j = 0; j < kd.M(); ++j)
                    if (kd.owns(d, j) != (j < L && j >= kd.first(d) && j < kd.first(d) + kd.width(d))) ++bad;
            }
            if (covered != L) ++bad;
        }
    if (bad == 0) printf("ok %ld\n", checked);
    return bad;
}
