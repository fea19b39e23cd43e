// Integers from their residues modulo several plaintext moduli (Chinese
// remainder theorem): the network evaluated once per modulus t_i yields each
// output mod t_i, and these combine into the exact signed integer as long as
// M = prod t_i exceeds twice its magnitude (the plaintext moduli of the
// CIFAR network are combined this way in Sec. 4.4).
//
// Per value, on the device: Garner's mixed-radix digits
//   v_0 = r_0,  v_i = (r_i - (v_0 + v_1 t_0 + ... + v_{i-1} t_0..t_{i-2})) (t_0..t_{i-1})^-1  mod t_i,
// then X = v_0 + t_0 (v_1 + t_1 (v_2 + ...)) in 32-bit limbs, and X - M when
// X > (M - 1) / 2.  The result is written as little-endian two's complement
// 64-bit words.
#include <vector>

#include "lola_internal.hpp"

namespace lola {

constexpr uint32_t CRT_MAXK = 16;
constexpr uint32_t CRT_MAXW = 16;   // 32-bit limbs of the result (8 output words)

struct CrtConst {
    uint32_t k, limbs;
    uint32_t t[CRT_MAXK];
    uint32_t inv[CRT_MAXK];              // (t_0 .. t_{i-1})^-1 mod t_i
    uint32_t tmod[CRT_MAXK][CRT_MAXK];   // t_l mod t_i
    uint32_t M[CRT_MAXW], halfM[CRT_MAXW];
};

struct CrtIn {
    const int64_t *r[CRT_MAXK];
};

__global__ void crt_combine_kernel(CrtIn in, CrtConst c, uint32_t n, int64_t *__restrict__ out) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t v[CRT_MAXK];
    for (uint32_t i = 0; i < c.k; ++i) {
        const int64_t ti = c.t[i];
        int64_t r = in.r[i][s] % ti;
        if (r < 0) r += ti;
        uint64_t acc = 0;   // v_0 + v_1 t_0 + ... mod t_i, by Horner from the top
        for (uint32_t l = i; l-- > 0;) acc = (acc * c.tmod[i][l] + v[l]) % (uint64_t)ti;
        uint64_t d = ((uint64_t)r + (uint64_t)ti - acc) % (uint64_t)ti;
        v[i] = (uint32_t)(d * c.inv[i] % (uint64_t)ti);
    }
    uint32_t x[CRT_MAXW];
    for (uint32_t w = 0; w < CRT_MAXW; ++w) x[w] = 0;
    for (uint32_t i = c.k; i-- > 0;) {   // X = X t_i + v_i
        uint64_t carry = v[i];
        for (uint32_t w = 0; w < c.limbs; ++w) {
            const uint64_t p = (uint64_t)x[w] * c.t[i] + carry;
            x[w] = (uint32_t)p;
            carry = p >> 32;
        }
    }
    bool greater = false;   // X > (M - 1) / 2
    for (uint32_t w = c.limbs; w-- > 0;) {
        if (x[w] != c.halfM[w]) {
            greater = x[w] > c.halfM[w];
            break;
        }
    }
    if (greater) {   // X - M, two's complement across all limbs
        uint64_t borrow = 0;
        for (uint32_t w = 0; w < c.limbs; ++w) {
            const uint64_t d = (uint64_t)x[w] - c.M[w] - borrow;
            x[w] = (uint32_t)d;
            borrow = (d >> 63) & 1;
        }
    }
    int64_t *o = out + (size_t)s * (c.limbs / 2);
    for (uint32_t w = 0; w < c.limbs; w += 2) o[w / 2] = (int64_t)(((uint64_t)x[w + 1] << 32) | x[w]);
}

static uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t r = a % b;
        a = b;
        b = r;
    }
    return a;
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_crt_combine(const int64_t *const *residues_dev, const uint32_t *moduli, uint32_t k, uint32_t n,
                     int64_t *out_dev, uint32_t words, lola_stream stream) {
    if (!residues_dev || !moduli || (n && !out_dev)) return set_error(LOLA_E_INVAL, "null argument");
    if (k < 1 || k > CRT_MAXK) return set_error(LOLA_E_INVAL, "between 1 and 16 moduli");
    if (words < 1 || 2 * words > CRT_MAXW) return set_error(LOLA_E_INVAL, "between 1 and 8 output words");
    CrtConst c{};
    c.k = k;
    c.limbs = 2 * words;
    for (uint32_t i = 0; i < k; ++i) {
        if (moduli[i] < 2 || moduli[i] >= (1u << 26)) return set_error(LOLA_E_INVAL, "moduli must lie in [2, 2^26)");
        if (!residues_dev[i]) return set_error(LOLA_E_INVAL, "null residue array");
        for (uint32_t l = 0; l < i; ++l)
            if (gcd64(moduli[i], moduli[l]) != 1) return set_error(LOLA_E_INVAL, "moduli must be pairwise coprime");
        c.t[i] = moduli[i];
    }
    // M = prod t_i in 32-bit limbs; the signed result needs M < 2^(64 words)
    std::vector<uint64_t> M(CRT_MAXW + 1, 0);
    M[0] = 1;
    for (uint32_t i = 0; i < k; ++i) {
        uint64_t carry = 0;
        for (uint32_t w = 0; w <= CRT_MAXW; ++w) {
            const uint64_t p = M[w] * moduli[i] + carry;
            M[w] = p & 0xffffffffu;
            carry = p >> 32;
        }
    }
    for (uint32_t w = c.limbs; w <= CRT_MAXW; ++w)
        if (M[w]) return set_error(LOLA_E_INVAL, "product of the moduli does not fit the output words");
    uint64_t rem = 0;   // halfM = (M - 1) / 2 (M is odd when every t_i is odd; floor either way)
    for (uint32_t w = c.limbs; w-- > 0;) {
        const uint64_t cur = (rem << 32) | (w == 0 ? M[0] - 1 : M[w]);
        c.halfM[w] = (uint32_t)(cur >> 1);
        rem = cur & 1;
        c.M[w] = (uint32_t)M[w];
    }
    for (uint32_t i = 0; i < k; ++i) {
        uint64_t prod = 1 % moduli[i];
        for (uint32_t l = 0; l < k; ++l) c.tmod[i][l] = moduli[l] % moduli[i];
        for (uint32_t l = 0; l < i; ++l) prod = prod * (moduli[l] % moduli[i]) % moduli[i];
        // inverse by the extended Euclidean algorithm (the moduli need not be prime)
        int64_t a = (int64_t)prod, m = moduli[i], x0 = 1, x1 = 0;
        while (m) {
            const int64_t q = a / m, t2 = a - q * m;
            a = m;
            m = t2;
            const int64_t tx = x0 - q * x1;
            x0 = x1;
            x1 = tx;
        }
        if (a != 1) return set_error(LOLA_E_INVAL, "moduli must be pairwise coprime");
        c.inv[i] = (uint32_t)(((x0 % (int64_t)moduli[i]) + moduli[i]) % moduli[i]);
    }
    if (n == 0) return LOLA_OK;
    CrtIn in{};
    for (uint32_t i = 0; i < k; ++i) in.r[i] = residues_dev[i];
    hipLaunchKernelGGL(crt_combine_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, in, c, n, out_dev);
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

}  // extern "C"
