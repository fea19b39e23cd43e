// Residue arithmetic modulo word-size primes q < 2^30 on 32-bit lanes.
//
// gfx950 has no fast 64-bit integer multiply, so every product is built from
// 32-bit multiplies:
//   - Shoup multiplication for a constant operand w with companion
//     w' = floor(w * 2^32 / q): a*w mod q in [0, 2q) for any a < 2^32, three
//     32-bit multiplies (twiddles, CRT constants, scalars);
//   - Montgomery reduction (R = 2^32) for variable x variable products, where
//     one side is usually stored premultiplied by R (keys, plaintexts);
//   - 64-bit accumulation of several products followed by one reduction
//     (key inner products).
// Lazily reduced values live in [0, 2q) or [0, 4q); q < 2^30 keeps 4q < 2^32.
#pragma once
#include <stdint.h>

#ifndef LOLA_HD
#include <hip/hip_runtime.h>
#define LOLA_HD __host__ __device__ __forceinline__
#endif

namespace lola {

// Loads and stores of one limb (or any buffer below 4 GiB) through a buffer
// resource: a scalar base and size plus a 32-bit lane offset.  Pointers read
// from job descriptors are generic, and plain indexing through them costs a
// flat access with 64-bit address arithmetic per element.  Accesses past the
// given size read 0 and drop the store instead of faulting.
#if defined(__HIP_DEVICE_COMPILE__)
struct GBuf {
    __amdgpu_buffer_rsrc_t r;
};
LOLA_HD GBuf gbuf(const uint32_t *base, uint32_t n_words) {
    return GBuf{__builtin_amdgcn_make_buffer_rsrc((void *)base, 0, (int)(n_words * 4u), 0x00020000)};
}
LOLA_HD uint32_t gld(GBuf b, uint32_t i) { return __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)(i << 2), 0, 0); }
LOLA_HD void gst(GBuf b, uint32_t i, uint32_t v) { __builtin_amdgcn_raw_buffer_store_b32(v, b.r, (int)(i << 2), 0, 0); }
// Four consecutive words at i (i a multiple of 4).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
LOLA_HD u32x4 gld4(GBuf b, uint32_t i) { return __builtin_amdgcn_raw_buffer_load_b128(b.r, (int)(i << 2), 0, 0); }
LOLA_HD void gst4(GBuf b, uint32_t i, u32x4 v) { __builtin_amdgcn_raw_buffer_store_b128(v, b.r, (int)(i << 2), 0, 0); }
#else
struct GBuf {
    uint32_t *p;
    uint32_t n;
};
LOLA_HD GBuf gbuf(const uint32_t *base, uint32_t n_words) { return GBuf{(uint32_t *)base, n_words}; }
LOLA_HD uint32_t gld(GBuf b, uint32_t i) { return i < b.n ? b.p[i] : 0u; }
LOLA_HD void gst(GBuf b, uint32_t i, uint32_t v) {
    if (i < b.n) b.p[i] = v;
}
struct u32x4 {
    uint32_t x, y, z, w;
};
LOLA_HD u32x4 gld4(GBuf b, uint32_t i) { return u32x4{gld(b, i), gld(b, i + 1), gld(b, i + 2), gld(b, i + 3)}; }
LOLA_HD void gst4(GBuf b, uint32_t i, u32x4 v) {
    gst(b, i, v.x);
    gst(b, i + 1, v.y);
    gst(b, i + 2, v.z);
    gst(b, i + 3, v.w);
}
#endif

// Per-modulus constants (one entry per prime of a context).
struct ModConst {
    uint32_t q;        // the prime
    uint32_t twoq;     // 2q
    uint32_t qneg_inv; // -q^{-1} mod 2^32 (Montgomery)
    uint32_t r_mod;    // 2^32 mod q
    uint32_t r2_mod;   // 2^64 mod q
    uint32_t r2_shoup; // Shoup companion of r2_mod
    uint32_t one_shoup;// floor(2^32 / q): Shoup companion of 1 (plain reduction)
    uint32_t ninv;     // N^{-1} mod q
    uint32_t ninv_shoup;
    uint32_t last_w;   // N^{-1} * psi^{-1}_{br}[1] mod q (last inverse stage)
    uint32_t last_w_shoup;
    uint32_t r_shoup;  // Shoup companion of r_mod
};

// A constant multiplier with its Shoup companion, loaded as one 64-bit word.
struct TwPair {
    uint32_t w, wp;
};

LOLA_HD uint32_t mulhi32(uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(a, b);
#else
    return (uint32_t)(((uint64_t)a * b) >> 32);
#endif
}

// a in [0, 2m) -> [0, m)
LOLA_HD uint32_t csub(uint32_t a, uint32_t m) {
    uint32_t d = a - m;
    return d < a ? d : a;  // unsigned: if a < m, d wraps above a
}

// Shoup: a * w mod q, result in [0, 2q), for any a < 2^32, w < q, wp = floor(w 2^32 / q).
LOLA_HD uint32_t shoup_lazy(uint32_t a, uint32_t w, uint32_t wp, uint32_t q) {
    uint32_t h = mulhi32(a, wp);
    return a * w - h * q;
}

LOLA_HD uint32_t shoup(uint32_t a, uint32_t w, uint32_t wp, uint32_t q) {
    return csub(shoup_lazy(a, w, wp, q), q);
}

// x mod q for any x < 2^32 (Shoup with w = 1).
LOLA_HD uint32_t reduce32(uint32_t x, uint32_t q, uint32_t one_shoup) {
    uint32_t h = mulhi32(x, one_shoup);
    return csub(x - h * q, q);
}

// Montgomery REDC of T = hi*2^32 + lo with T < 2q * 2^32: returns T * 2^-32 mod q in [0, 3q).
LOLA_HD uint32_t redc_lazy(uint32_t lo, uint32_t hi, uint32_t q, uint32_t qneg_inv) {
    uint32_t m = lo * qneg_inv;
    // (T + m q) / 2^32; the low words sum to 0 mod 2^32, carrying out iff lo != 0.
    return hi + mulhi32(m, q) + (lo != 0u ? 1u : 0u);
}

// a * b * 2^-32 mod q, a, b < 2^32 with a*b < 2q * 2^32; result in [0, q).
LOLA_HD uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t q, uint32_t qneg_inv) {
    uint32_t lo = a * b;
    uint32_t hi = mulhi32(a, b);
    uint32_t r = redc_lazy(lo, hi, q, qneg_inv);
    r = csub(r, 2 * q);
    return csub(r, q);
}

// 64-bit accumulator of products of residues, reduced once.
struct Acc64 {
    uint32_t lo, hi;
};

LOLA_HD void acc_mad(Acc64 &acc, uint32_t a, uint32_t b) {
    uint32_t plo = a * b;
    uint32_t phi = mulhi32(a, b);
    uint32_t nlo = acc.lo + plo;
    acc.hi += phi + (nlo < plo ? 1u : 0u);
    acc.lo = nlo;
}

// acc * 2^-32 mod q for any 64-bit acc (the hi word is reduced first so that
// the Montgomery step's input stays below 2q * 2^32).
LOLA_HD uint32_t acc_reduce_mont(const Acc64 &acc, const ModConst &c) {
    uint32_t hi = acc.hi - mulhi32(acc.hi, c.one_shoup) * c.q;  // [0, 2q)
    uint32_t r = redc_lazy(acc.lo, hi, c.q, c.qneg_inv);                          // [0, 3q)
    r = csub(r, 2 * c.q);
    return csub(r, c.q);
}

LOLA_HD uint32_t add_mod(uint32_t a, uint32_t b, uint32_t q) { return csub(a + b, q); }
LOLA_HD uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t q) { return csub(a + q - b, q); }

}  // namespace lola
