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
//
// Batched: any number of independent pairs, each with its own scratch.
#include "mrc.hpp"
#include "program.hpp"

namespace lola {

struct MulLayout {           // word offsets inside one job's scratch
    size_t Ac, Bx, Dq, Db, Oc, total;
};
static MulLayout mul_layout(size_t L, size_t nB, size_t N) {
    MulLayout m;
    m.Ac = 0;                       // [4][L][N]  inputs, coefficient form
    m.Bx = m.Ac + 4 * L * N;        // [4][nB][N] inputs extended to B
    m.Dq = m.Bx + 4 * nB * N;       // [3][L][N]  tensor in Q
    m.Db = m.Dq + 3 * L * N;        // [3][nB][N] tensor in B
    m.Oc = m.Db + 3 * nB * N;       // [3][L][N]  rounded result, coefficient form
    m.total = m.Oc + 3 * L * N;
    return m;
}

// Q -> B centred extension of one coefficient of one of the four inputs.
// grid (N/256, 4, jobs)
__global__ void tensor_extend_kernel(const MulJob *__restrict__ jobs, uint32_t N, size_t offAc, size_t offBx,
                                     const ModConst *__restrict__ mcs, const MrcConst *__restrict__ mrc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x, p = blockIdx.y;
    if (k >= N) return;
    const MulJob job = jobs[blockIdx.z];
    if (p >= 2 && job.a == job.b) return;   // a square: the second operand is the first
    const uint32_t *src = job.scr + offAc;
    uint32_t *dst = job.scr + offBx;
    const int L = (int)mrc->L, nB = (int)mrc->nB;
    uint32_t r[MAXL], v[MAXL];
    // every load issued unconditionally (limbs past L read limb L-1 again and
    // are zeroed after): a test per limb would wait for each load in turn
#pragma unroll
    for (int i = 0; i < MAXL; ++i) r[i] = src[((size_t)p * L + min(i, L - 1)) * N + k];
#pragma unroll
    for (int i = 0; i < MAXL; ++i) r[i] = i < L ? r[i] : 0;
    mrc_digits<MAXL>(r, v, L, mcs, mrc->invQ, mrc->invQp);
    const bool neg = mrc_greater<MAXL>(v, L, mrc->hQ);
    const ModConst *mb = mcs + L + mrc->K;   // the auxiliary primes
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
// grid (N/256, L + nB, jobs)
__global__ void tensor_product_kernel(const MulJob *__restrict__ jobs, uint32_t N, uint32_t L, uint32_t nB,
                                      size_t offBx, size_t offDq, size_t offDb,
                                      const ModConst *__restrict__ mcs, const ModConst *__restrict__ mbs) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x, l = blockIdx.y;
    if (k >= N) return;
    const MulJob job = jobs[blockIdx.z];
    uint32_t a0, a1, b0, b1;
    ModConst c;
    if (l < L) {
        c = mcs[l];
        const size_t o = (size_t)l * N + k, P1 = (size_t)L * N;
        a0 = job.a[o]; a1 = job.a[P1 + o]; b0 = job.b[o]; b1 = job.b[P1 + o];
    } else {
        const uint32_t j = l - L;
        c = mbs[j];
        const uint32_t *ext = job.scr + offBx;
        const size_t o = (size_t)j * N + k, PB = (size_t)nB * N, ob = job.a == job.b ? o : 2 * PB + o;
        a0 = ext[o]; a1 = ext[PB + o]; b0 = ext[ob]; b1 = ext[PB + ob];
    }
    const uint32_t a0m = shoup(a0, c.r_mod, c.r_shoup, c.q), a1m = shoup(a1, c.r_mod, c.r_shoup, c.q);
    const uint32_t d0 = mont_mul(a0m, b0, c.q, c.qneg_inv);
    const uint32_t d1 = add_mod(mont_mul(a0m, b1, c.q, c.qneg_inv), mont_mul(a1m, b0, c.q, c.qneg_inv), c.q);
    const uint32_t d2 = mont_mul(a1m, b1, c.q, c.qneg_inv);
    if (l < L) {
        uint32_t *dq = job.scr + offDq;
        const size_t o = (size_t)l * N + k, P1 = (size_t)L * N;
        dq[o] = d0; dq[P1 + o] = d1; dq[2 * P1 + o] = d2;
    } else {
        uint32_t *db = job.scr + offDb;
        const size_t o = (size_t)(l - L) * N + k, PB = (size_t)nB * N;
        db[o] = d0; db[PB + o] = d1; db[2 * PB + o] = d2;
    }
}

// round(t d / Q) for one coefficient of output polynomial p.
// grid (N/256, 3, jobs)
__global__ void tensor_round_kernel(const MulJob *__restrict__ jobs, uint32_t N, size_t offDq, size_t offDb,
                                    size_t offOc, const ModConst *__restrict__ mcs,
                                    const MrcConst *__restrict__ mrc) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x, p = blockIdx.y;
    if (k >= N) return;
    const MulJob job = jobs[blockIdx.z];
    const uint32_t *dq = job.scr + offDq, *db = job.scr + offDb;
    uint32_t *out = job.scr + offOc;
    const int L = (int)mrc->L, nB = (int)mrc->nB;
    uint32_t r[MAXL], v[MAXL], tdb[MAXB];
    // all loads first, unconditionally (limbs past L or nB read the last one
    // again and are ignored): a test per limb would wait for each load in turn
#pragma unroll
    for (int i = 0; i < MAXL; ++i) r[i] = dq[((size_t)p * L + min(i, L - 1)) * N + k];
#pragma unroll
    for (int j = 0; j < MAXB; ++j) tdb[j] = db[((size_t)p * nB + min(j, nB - 1)) * N + k];
#pragma unroll
    for (int i = 0; i < MAXL; ++i) r[i] = i < L ? shoup(r[i], mrc->tq[i], mrc->tqp[i], mcs[i].q) : 0;
    mrc_digits<MAXL>(r, v, L, mcs, mrc->invQ, mrc->invQp);   // digits of R = t d mod Q
    const uint32_t carry = mrc_greater<MAXL>(v, L, mrc->hQ) ? 1u : 0u;
    const ModConst *mb = mcs + L + mrc->K;   // the auxiliary primes
    uint32_t z[MAXB], w[MAXB];
#pragma unroll
    for (int j = 0; j < MAXB; ++j) {
        if (j < nB) {
            const uint32_t bq = mb[j].q;
            const uint32_t Rb = mrc_eval<MAXL>(v, L, mrc->wQb[j], mrc->wQbp[j], bq);
            const uint32_t td = shoup(tdb[j], mrc->tb[j], mrc->tbp[j], bq);
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

size_t mul_scratch_words(const lola_ctx *ctx) { return mul_layout(ctx->L, ctx->nB, ctx->N).total; }

// Algorithmic cost per pair (a square extends and reads its operand once):
//   extend   per input polynomial: L limbs in, nB out; Garner digits over Q
//            (L(L-1)/2 products and subtracts), the sign test, and nB
//            evaluations of L digits (a product and an add each)
//   product  per limb of Q u B: the operands in, three limbs out; two Shoup
//            and four Montgomery products and an add a coefficient
//   round    per output polynomial: L + nB limbs in, L out; t d mod Q's
//            digits, per b in B the evaluation, scaling and carry, the digits
//            over B, and per q in Q the evaluation and sign correction
int launch_mul_stage(lola_ctx *ctx, uint32_t stage, const MulJob *d, uint32_t n, uint64_t n_squares,
                     hipStream_t s) {
    const uint32_t N = ctx->N, L = ctx->L, nB = ctx->nB;
    const MulLayout ml = mul_layout(L, nB, N);
    const double dN = N, dL = L, dB = nB, polys = 4.0 * n - 2.0 * n_squares;
    const double M = COST_MUL, A = COST_ADD;
    if (stage == LK_MUL_EXTEND)
        LOLA_TIMED(ctx, s, KID_TENSOR_EXTEND, n, polys * 4 * dN * (dL + dB),
                   polys * dN * (dL * (dL - 1) / 2 * (M + A) + dL + dB * dL * (M + A)),
                   hipLaunchKernelGGL(tensor_extend_kernel, dim3(N / 256, 4, n), dim3(256), 0, s, d, N, ml.Ac,
                                      ml.Bx, ctx->d_mc, ctx->d_mrc));
    else if (stage == LK_MUL_PRODUCT)
        LOLA_TIMED(ctx, s, KID_TENSOR_PRODUCT, n, (polys + 3.0 * n) * 4 * dN * (dL + dB),
                   n * dN * (dL + dB) * (6 * M + A),
                   hipLaunchKernelGGL(tensor_product_kernel, dim3(N / 256, L + nB, n), dim3(256), 0, s, d, N, L,
                                      nB, ml.Bx, ml.Dq, ml.Db, ctx->d_mc, ctx->d_mc + ctx->idxB(0)));
    else
        LOLA_TIMED(ctx, s, KID_TENSOR_ROUND, n, 3.0 * n * 4 * dN * (2 * dL + dB),
                   3.0 * n * dN * (dL * M + dL * (dL - 1) / 2 * (M + A) + dL + dB * (dL * (M + A) + 2 * M + 2 * A) +
                                   dB * (dB - 1) / 2 * (M + A) + dB + dL * (dB * (M + A) + A)),
                   hipLaunchKernelGGL(tensor_round_kernel, dim3(N / 256, 3, n), dim3(256), 0, s, d, N, ml.Dq, ml.Db,
                                      ml.Oc, ctx->d_mc, ctx->d_mrc));
    LOLA_HIP(hipGetLastError());
    return LOLA_OK;
}

void program_mul(const lola_ctx *ctx, Program &p, const std::vector<MulJob> &pairs, uint32_t *scratch,
                 uint32_t chunk) {
    const size_t N = ctx->N, L = ctx->L, nB = ctx->nB, P1 = L * N;
    const MulLayout ml = mul_layout(L, nB, N);
    for (size_t off = 0; off < pairs.size(); off += chunk) {
        const size_t m = std::min<size_t>(chunk, pairs.size() - off);
        std::vector<MulJob> jobs(m);
        std::vector<NttJob> n1, n2, n3, n4;
        for (size_t k = 0; k < m; ++k) {
            MulJob j = pairs[off + k];
            j.scr = scratch + ml.total * k;
            jobs[k] = j;
            // a square (a == b) transforms and extends its operand once; the
            // product kernel reads the first operand's extension for both
            const int nops = j.a == j.b ? 2 : 4;
            const uint32_t *srcs[4] = {j.a, j.a + P1, j.b, j.b + P1};
            for (int q = 0; q < nops; ++q)
                for (uint32_t i = 0; i < L; ++i)
                    n1.push_back(NttJob{srcs[q] + i * N, j.scr + ml.Ac + (q * L + i) * N, i, NTT_INVERSE});
            for (int q = 0; q < nops; ++q)
                for (uint32_t b = 0; b < nB; ++b) {
                    uint32_t *x = j.scr + ml.Bx + (q * nB + b) * N;
                    n2.push_back(NttJob{x, x, ctx->idxB(b), 0});
                }
            for (int q = 0; q < 3; ++q) {
                for (uint32_t i = 0; i < L; ++i) {
                    uint32_t *x = j.scr + ml.Dq + (q * L + i) * N;
                    n3.push_back(NttJob{x, x, i, NTT_INVERSE});
                }
                for (uint32_t b = 0; b < nB; ++b) {
                    uint32_t *x = j.scr + ml.Db + (q * nB + b) * N;
                    n3.push_back(NttJob{x, x, ctx->idxB(b), NTT_INVERSE});
                }
                for (uint32_t i = 0; i < L; ++i)
                    n4.push_back(NttJob{j.scr + ml.Oc + (q * L + i) * N, j.out3 + (q * L + i) * N, i, 0});
            }
        }
        const size_t dj = p.put(jobs);
        Launch ml_launch{LK_MUL_EXTEND, (uint32_t)m, dj};
        launch_aux(jobs, ml_launch.aux);
        p.launch(LK_NTT, n1);
        p.launches.push_back(ml_launch);
        p.launch(LK_NTT, n2);
        ml_launch.kind = LK_MUL_PRODUCT;
        p.launches.push_back(ml_launch);
        p.launch(LK_NTT, n3);
        ml_launch.kind = LK_MUL_ROUND;
        p.launches.push_back(ml_launch);
        p.launch(LK_NTT, n4);
    }
}

int mul_batch(lola_ctx *ctx, uint32_t n, const uint32_t *const *a, const uint32_t *const *b,
              uint32_t *const *out3, hipStream_t s) {
    constexpr uint32_t CHUNK = 8;   // bounds one blob to a descriptor-ring slab
    for (uint32_t off = 0; off < n; off += CHUNK) {
        const uint32_t m = std::min(CHUNK, n - off);
        std::vector<MulJob> pairs(m);
        for (uint32_t k = 0; k < m; ++k) {
            if (!a[off + k] || !b[off + k] || !out3[off + k]) return set_error(LOLA_E_INVAL, "null pointer in batch");
            if (out3[off + k] == a[off + k] || out3[off + k] == b[off + k])
                return set_error(LOLA_E_INVAL, "product output may not alias an input");
            pairs[k] = MulJob{a[off + k], b[off + k], out3[off + k], nullptr};
        }
        void *buf = nullptr;
        int rc = scratch_get(ctx, mul_scratch_words(ctx) * m * 4, &buf);
        if (rc) return rc;
        Program p;
        program_mul(ctx, p, pairs, (uint32_t *)buf, m);
        if ((rc = program_run_now(ctx, p, s))) return rc;
    }
    return LOLA_OK;
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_mul(lola_ctx *ctx, const uint32_t *a, const uint32_t *b, uint32_t *out3, lola_stream stream) {
    if (!ctx || !a || !b || !out3) return set_error(LOLA_E_INVAL, "null argument");
    return mul_batch(ctx, 1, &a, &b, &out3, (hipStream_t)stream);
}

}  // extern "C"
