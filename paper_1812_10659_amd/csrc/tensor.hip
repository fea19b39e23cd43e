// Exact ciphertext x ciphertext product: d_j = round(t (a (x) b)_j / Q) mod Q.
//
// The tensor of the centred lifts is an integer polynomial whose coefficients
// exceed Q, so it is computed in the extended basis Q u B (B: auxiliary
// primes, product B > 2 t N Q).  The inputs are extended from Q to B exactly
// (mixed-radix digits, centred by comparing with (Q-1)/2), the three products
// are formed limb by limb in the NTT domain, and the rounding is done without
// any floating-point estimate:
//   R = (t d) mod Q from its residues; floor(t d / Q) = (t d - R) / Q, which
//   is computed modulo every b in B; round adds [R > (Q-1)/2] (no ties: Q odd).
// The result Z (|Z| < B/2) is then converted from B back to Q, again through
// its mixed-radix digits, and centred.
#include "lola_internal.hpp"
#include "mrc.hpp"

namespace lola {

// Q -> B centred extension of one coefficient of one polynomial.
// src: [L][N] coefficient residues of 4 polynomials; dst: [nB][N] per poly.
__global__ void tensor_extend_kernel(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, uint32_t N,
                                     const ModConst *__restrict__ mcs, const MrcConst *__restrict__ mrc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x, p = blockIdx.y;
    if (k >= N) return;
    const int L = (int)mrc->L, nB = (int)mrc->nB;
    uint32_t r[MAXL], v[MAXL];
#pragma unroll
    for (int i = 0; i < MAXL; ++i) r[i] = i < L ? src[((size_t)p * L + i) * N + k] : 0;
    mrc_digits<MAXL>(r, v, L, mcs, mrc->invQ, mrc->invQp);
    const bool neg = mrc_greater<MAXL>(v, L, mrc->hQ);
    const ModConst *mb = mcs + L + 1;
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
        if (j < nB) {
            const uint32_t bq = mb[j].q;
            uint32_t x = mrc_eval<MAXL>(v, L, mrc->wQb[j], mrc->wQbp[j], bq);
            if (neg) x = sub_mod(x, mrc->Qb[j], bq);
            dst[((size_t)p * nB + j) * N + k] = x;
        }
    }
}

// d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 on limb l of Q u B (NTT domain).
// grid (N/256, L + nB)
__global__ void tensor_product_kernel(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                                      const uint32_t *__restrict__ ext, uint32_t *__restrict__ dq,
                                      uint32_t *__restrict__ db, uint32_t N, uint32_t L, uint32_t nB,
                                      const ModConst *__restrict__ mcs) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x, l = blockIdx.y;
    if (k >= N) return;
    uint32_t a0, a1, b0, b1;
    ModConst c;
    if (l < L) {
        c = mcs[l];
        const size_t o = (size_t)l * N + k, P1 = (size_t)L * N;
        a0 = a[o]; a1 = a[P1 + o]; b0 = b[o]; b1 = b[P1 + o];
    } else {
        const uint32_t j = l - L;
        c = mcs[L + 1 + j];
        const size_t o = (size_t)j * N + k, PB = (size_t)nB * N;
        a0 = ext[o]; a1 = ext[PB + o]; b0 = ext[2 * PB + o]; b1 = ext[3 * PB + o];
    }
    const uint32_t a0m = shoup(a0, c.r_mod, c.r_shoup, c.q), a1m = shoup(a1, c.r_mod, c.r_shoup, c.q);
    const uint32_t d0 = mont_mul(a0m, b0, c.q, c.qneg_inv);
    const uint32_t d1 = add_mod(mont_mul(a0m, b1, c.q, c.qneg_inv), mont_mul(a1m, b0, c.q, c.qneg_inv), c.q);
    const uint32_t d2 = mont_mul(a1m, b1, c.q, c.qneg_inv);
    if (l < L) {
        const size_t o = (size_t)l * N + k, P1 = (size_t)L * N;
        dq[o] = d0; dq[P1 + o] = d1; dq[2 * P1 + o] = d2;
    } else {
        const size_t o = (size_t)(l - L) * N + k, PB = (size_t)nB * N;
        db[o] = d0; db[PB + o] = d1; db[2 * PB + o] = d2;
    }
}

// round(t d / Q) for one coefficient of output polynomial p; dq [3][L][N],
// db [3][nB][N] coefficient residues; out [3][L][N] coefficient residues.
__global__ void tensor_round_kernel(const uint32_t *__restrict__ dq, const uint32_t *__restrict__ db,
                                    uint32_t *__restrict__ out, uint32_t N, const ModConst *__restrict__ mcs,
                                    const MrcConst *__restrict__ mrc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x, p = blockIdx.y;
    if (k >= N) return;
    const int L = (int)mrc->L, nB = (int)mrc->nB;
    uint32_t r[MAXL], v[MAXL];
#pragma unroll
    for (int i = 0; i < MAXL; ++i)
        r[i] = i < L ? shoup(dq[((size_t)p * L + i) * N + k], mrc->tq[i], mrc->tqp[i], mcs[i].q) : 0;
    mrc_digits<MAXL>(r, v, L, mcs, mrc->invQ, mrc->invQp);   // digits of R = t d mod Q
    const uint32_t carry = mrc_greater<MAXL>(v, L, mrc->hQ) ? 1u : 0u;
    const ModConst *mb = mcs + L + 1;
    uint32_t z[MAXB], w[MAXB];
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
        if (j < nB) {
            const uint32_t bq = mb[j].q;
            const uint32_t Rb = mrc_eval<MAXL>(v, L, mrc->wQb[j], mrc->wQbp[j], bq);
            const uint32_t td = shoup(db[((size_t)p * nB + j) * N + k], mrc->tb[j], mrc->tbp[j], bq);
            uint32_t y = shoup(sub_mod(td, Rb, bq), mrc->Qinvb[j], mrc->Qinvbp[j], bq);
            z[j] = add_mod(y, carry, bq);
        } else {
            z[j] = 0;
        }
    }
    mrc_digits<MAXB>(z, w, nB, mb, mrc->invB, mrc->invBp);     // digits of Z over B
    const bool neg = mrc_greater<MAXB>(w, nB, mrc->hB);
#pragma unroll
    for (int i = 0; i < MAXL; ++i) {
        if (i < L) {
            const uint32_t q = mcs[i].q;
            uint32_t x = mrc_eval<MAXB>(w, nB, mrc->wBq[i], mrc->wBqp[i], q);
            if (neg) x = sub_mod(x, mrc->Bq[i], q);
            out[((size_t)p * L + i) * N + k] = x;
        }
    }
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_mul(lola_ctx *ctx, const uint32_t *a, const uint32_t *b, uint32_t *out3, lola_stream stream) {
    if (!ctx || !a || !b || !out3) return set_error(LOLA_E_INVAL, "null argument");
    if (out3 == a || out3 == b) return set_error(LOLA_E_INVAL, "lola_mul output may not alias an input");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = ctx->N, L = ctx->L, nB = ctx->nB;
    // Ac [4][L][N] | Bx [4][nB][N] | Dq [3][L][N] | Db [3][nB][N] | Oc [3][L][N]
    const size_t words = (4 * L + 4 * nB + 3 * L + 3 * nB + 3 * L) * N;
    void *buf = nullptr;
    int rc = scratch_get(ctx, words * 4, &buf);
    if (rc) return rc;
    uint32_t *Ac = (uint32_t *)buf, *Bx = Ac + 4 * L * N, *Dq = Bx + 4 * nB * N, *Db = Dq + 3 * L * N,
             *Oc = Db + 3 * nB * N;
    const size_t P1 = L * N;
    std::vector<NttJob> jobs;
    const uint32_t *srcs[4] = {a, a + P1, b, b + P1};
    for (int p = 0; p < 4; ++p)
        for (uint32_t i = 0; i < L; ++i)
            jobs.push_back(NttJob{srcs[p] + i * N, Ac + (p * L + i) * N, i, NTT_INVERSE});
    if ((rc = launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), s))) return rc;
    hipLaunchKernelGGL(tensor_extend_kernel, dim3((unsigned)(N / 256), 4), dim3(256), 0, s, Ac, Bx, (uint32_t)N,
                       ctx->d_mc, ctx->d_mrc);
    LOLA_HIP(hipGetLastError());
    jobs.clear();
    for (int p = 0; p < 4; ++p)
        for (uint32_t j = 0; j < nB; ++j)
            jobs.push_back(NttJob{Bx + (p * nB + j) * N, Bx + (p * nB + j) * N, ctx->idxB(j), 0});
    if ((rc = launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), s))) return rc;
    hipLaunchKernelGGL(tensor_product_kernel, dim3((unsigned)(N / 256), (unsigned)(L + nB)), dim3(256), 0, s, a, b,
                       Bx, Dq, Db, (uint32_t)N, (uint32_t)L, (uint32_t)nB, ctx->d_mc);
    LOLA_HIP(hipGetLastError());
    jobs.clear();
    for (int p = 0; p < 3; ++p) {
        for (uint32_t i = 0; i < L; ++i)
            jobs.push_back(NttJob{Dq + (p * L + i) * N, Dq + (p * L + i) * N, i, NTT_INVERSE});
        for (uint32_t j = 0; j < nB; ++j)
            jobs.push_back(NttJob{Db + (p * nB + j) * N, Db + (p * nB + j) * N, ctx->idxB(j), NTT_INVERSE});
    }
    if ((rc = launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), s))) return rc;
    hipLaunchKernelGGL(tensor_round_kernel, dim3((unsigned)(N / 256), 3), dim3(256), 0, s, Dq, Db, Oc, (uint32_t)N,
                       ctx->d_mc, ctx->d_mrc);
    LOLA_HIP(hipGetLastError());
    jobs.clear();
    for (int p = 0; p < 3; ++p)
        for (uint32_t i = 0; i < L; ++i) jobs.push_back(NttJob{Oc + (p * L + i) * N, out3 + (p * L + i) * N, i, 0});
    return launch_ntt_jobs(ctx, jobs.data(), (int)jobs.size(), s);
}

}  // extern "C"
