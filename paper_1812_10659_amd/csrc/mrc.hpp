// Exact mixed-radix (Garner) conversions between RNS bases, per coefficient.
//
// A residue vector (x mod q_0, ..., x mod q_{n-1}) of an integer X in [0, Q)
// has unique digits v_k in [0, q_k) with X = v_0 + v_1 q_0 + v_2 q_0 q_1 + ...
// From the digits, X mod any other modulus m is sum_k v_k (q_0...q_{k-1} mod m)
// and X > (Q-1)/2 is a lexicographic comparison with the digits of (Q-1)/2.
// Everything is integer arithmetic with precomputed constants, so the results
// are exact (no floating-point estimate of the CRT overflow).
#pragma once
#include "lola_internal.hpp"

namespace lola {

// Digits over the first n primes of a basis.  inv[i][k] = p_k^-1 mod p_i.
template <int MAXN>
__device__ __forceinline__ void mrc_digits(const uint32_t (&r)[MAXN], uint32_t (&v)[MAXN], int n,
                                           const ModConst *__restrict__ mcs, const uint32_t (*inv)[MAXN],
                                           const uint32_t (*invp)[MAXN]) {
#pragma unroll
    for (int i = 0; i < MAXN; ++i) {
        if (i < n) {
            const ModConst &c = mcs[i];
            uint32_t u = r[i];
#pragma unroll
            for (int k = 0; k < MAXN; ++k) {
                if (k < i) {
                    uint32_t vk = reduce32(v[k], c.q, c.one_shoup);
                    u = sub_mod(u, vk, c.q);
                    u = shoup(u, inv[i][k], invp[i][k], c.q);
                }
            }
            v[i] = u;
        } else {
            v[i] = 0;
        }
    }
}

// sum_k v_k W_k mod m, with W_k (mod m) Shoup pairs in w[k], wp[k].
template <int MAXN>
__device__ __forceinline__ uint32_t mrc_eval(const uint32_t (&v)[MAXN], int n, const uint32_t *w,
                                             const uint32_t *wp, uint32_t m) {
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < MAXN; ++k)
        if (k < n) acc = add_mod(acc, shoup(v[k], w[k], wp[k], m), m);
    return acc;
}

// X > H where h holds the digits of H = (Q-1)/2.
template <int MAXN>
__device__ __forceinline__ bool mrc_greater(const uint32_t (&v)[MAXN], int n, const uint32_t *h) {
    bool gt = false, decided = false;
#pragma unroll
    for (int k = MAXN - 1; k >= 0; --k) {
        if (k < n && !decided) {
            if (v[k] != h[k]) {
                gt = v[k] > h[k];
                decided = true;
            }
        }
    }
    return gt;
}

}  // namespace lola
