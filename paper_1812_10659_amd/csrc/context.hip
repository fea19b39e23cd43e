// Context creation: parameter checks, NTT tables, exact mixed-radix constants.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>

#include "lola_internal.hpp"

namespace lola {

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int check_hip(hipError_t e, const char *what) {
    return set_error(LOLA_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)((unsigned __int128)a * b % m);
}
uint64_t powmod_host(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod_host(r, a, m);
        a = mulmod_host(a, a, m);
        e >>= 1;
    }
    return r;
}
uint64_t invmod_host(uint64_t a, uint64_t m) { return powmod_host(a % m, m - 2, m); }

static bool is_prime_u32(uint64_t n) {
    if (n < 2) return false;
    for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull}) {
        if (n % p == 0) return n == p;
    }
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; ++s; }
    for (uint64_t a : {2ull, 7ull, 61ull}) {  // deterministic below 2^32
        uint64_t x = powmod_host(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod_host(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

static uint32_t bitrev(uint32_t x, uint32_t bits) {
    uint32_t r = 0;
    for (uint32_t b = 0; b < bits; ++b)
        if (x & (1u << b)) r |= 1u << (bits - 1 - b);
    return r;
}

// Smallest primitive 2N-th root of unity mod m: all of them are the odd powers
// of any one, so take one and scan its N odd powers.
static uint64_t smallest_root_2n(uint64_t m, uint32_t N) {
    uint64_t e = (m - 1) / (2ull * N), psi0 = 0;
    for (uint64_t x = 2; x < m && !psi0; ++x) {
        uint64_t r = powmod_host(x, e, m);
        if (powmod_host(r, N, m) == m - 1) psi0 = r;
    }
    uint64_t best = psi0, cur = psi0, sq = mulmod_host(psi0, psi0, m);
    for (uint32_t k = 1; k < N; ++k) {
        cur = mulmod_host(cur, sq, m);
        best = std::min(best, cur);
    }
    return best;
}

static double cap_log2(uint32_t N) {
    switch (N) {
        case 1024: return 27; case 2048: return 54; case 4096: return 109;
        case 8192: return 218; case 16384: return 438; default: return 0;
    }
}

int scratch_get(lola_ctx *ctx, size_t bytes, void **out) {
    if (bytes > ctx->scratch_bytes) {
        if (ctx->d_scratch) {
            LOLA_HIP(hipDeviceSynchronize());
            LOLA_HIP(hipFree(ctx->d_scratch));
            ctx->d_scratch = nullptr;
            ctx->scratch_bytes = 0;
        }
        size_t want = std::max(bytes, (size_t)1 << 20);
        if (hipMalloc(&ctx->d_scratch, want) != hipSuccess)
            return set_error(LOLA_E_NOMEM, "scratch allocation of " + std::to_string(want) + " bytes failed");
        ctx->scratch_bytes = want;
    }
    *out = ctx->d_scratch;
    return LOLA_OK;
}

int desc_upload(lola_ctx *ctx, const void *host, size_t bytes, hipStream_t s, void **dev) {
    const size_t SL = lola_ctx::RING_SLAB;
    if (bytes > SL) return set_error(LOLA_E_INVAL, "descriptor batch too large (split the batch)");
    if (!ctx->h_ring) {
        LOLA_HIP(hipHostMalloc((void **)&ctx->h_ring, SL * lola_ctx::RING_SLABS, hipHostMallocDefault));
        LOLA_HIP(hipMalloc((void **)&ctx->d_ring, SL * lola_ctx::RING_SLABS));
        for (int i = 0; i < lola_ctx::RING_SLABS; ++i)
            LOLA_HIP(hipEventCreateWithFlags(&ctx->ring_ev[i], hipEventDisableTiming));
        ctx->ring_off = 0;
    }
    size_t off = (ctx->ring_off + 255) & ~(size_t)255;
    size_t slab = ctx->ring_off / SL;
    if (off + bytes > (slab + 1) * SL) {
        // leave this slab: mark the point after which it is free, move on
        LOLA_HIP(hipEventRecord(ctx->ring_ev[slab], s));
        ctx->ring_ev_valid[slab] = true;
        slab = (slab + 1) % lola_ctx::RING_SLABS;
        off = slab * SL;
        if (ctx->ring_ev_valid[slab]) {
            LOLA_HIP(hipEventSynchronize(ctx->ring_ev[slab]));
            ctx->ring_ev_valid[slab] = false;
        }
    }
    memcpy(ctx->h_ring + off, host, bytes);
    LOLA_HIP(hipMemcpyAsync(ctx->d_ring + off, ctx->h_ring + off, bytes, hipMemcpyHostToDevice, s));
    ctx->ring_off = off + bytes;
    *dev = ctx->d_ring + off;
    return LOLA_OK;
}

// Garner digits of x (residues r[i] mod m[i]) on the host.
static std::vector<uint64_t> mrc_host(const std::vector<uint64_t> &r, const std::vector<uint64_t> &m) {
    std::vector<uint64_t> v(r.size());
    for (size_t i = 0; i < r.size(); ++i) {
        uint64_t u = r[i] % m[i];
        for (size_t k = 0; k < i; ++k) {
            u = (u + m[i] - v[k] % m[i]) % m[i];
            u = mulmod_host(u, invmod_host(m[k] % m[i], m[i]), m[i]);
        }
        v[i] = u;
    }
    return v;
}

static int build_tables(lola_ctx *ctx) {
    const uint32_t N = ctx->N, np = ctx->nprimes();
    std::vector<TwPair> tw((size_t)np * N), itw(tw.size());
    ctx->mc_host.assign(np, ModConst{});
    for (uint32_t p = 0; p < np; ++p) {
        const uint64_t q = ctx->primes[p];
        const uint64_t psi = smallest_root_2n(q, N), ipsi = invmod_host(psi, q);
        // powers by bit-reversed index
        std::vector<uint64_t> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (uint32_t k = 1; k < N; ++k) {
            pw[k] = mulmod_host(pw[k - 1], psi, q);
            ipw[k] = mulmod_host(ipw[k - 1], ipsi, q);
        }
        for (uint32_t k = 0; k < N; ++k) {
            uint32_t b = bitrev(k, ctx->logN);
            tw[(size_t)p * N + k] = TwPair{(uint32_t)pw[b], shoup_companion((uint32_t)pw[b], (uint32_t)q)};
            itw[(size_t)p * N + k] = TwPair{(uint32_t)ipw[b], shoup_companion((uint32_t)ipw[b], (uint32_t)q)};
        }
        ModConst &c = ctx->mc_host[p];
        c.q = (uint32_t)q;
        c.twoq = (uint32_t)(2 * q);
        uint32_t inv = 1;  // Newton: inv = q^-1 mod 2^32
        for (int i = 0; i < 5; ++i) inv *= 2u - (uint32_t)q * inv;
        c.qneg_inv = 0u - inv;
        c.r_mod = (uint32_t)(((uint64_t)1 << 32) % q);
        c.r2_mod = (uint32_t)mulmod_host(c.r_mod, c.r_mod, q);
        c.r2_shoup = shoup_companion(c.r2_mod, (uint32_t)q);
        c.r_shoup = shoup_companion(c.r_mod, (uint32_t)q);
        c.one_shoup = (uint32_t)((((uint64_t)1) << 32) / q);
        uint64_t ninv = invmod_host(N, q);
        c.ninv = (uint32_t)ninv;
        c.ninv_shoup = shoup_companion(c.ninv, (uint32_t)q);
        c.last_w = (uint32_t)mulmod_host(ninv, itw[(size_t)p * N + 1].w, q);
        c.last_w_shoup = shoup_companion(c.last_w, (uint32_t)q);
    }
    size_t tb = tw.size() * sizeof(TwPair);
    LOLA_HIP(hipMalloc(&ctx->d_tw, tb));
    LOLA_HIP(hipMalloc(&ctx->d_itw, tb));
    LOLA_HIP(hipMemcpy(ctx->d_tw, tw.data(), tb, hipMemcpyHostToDevice));
    LOLA_HIP(hipMemcpy(ctx->d_itw, itw.data(), tb, hipMemcpyHostToDevice));
    LOLA_HIP(hipMalloc(&ctx->d_mc, np * sizeof(ModConst)));
    LOLA_HIP(hipMemcpy(ctx->d_mc, ctx->mc_host.data(), np * sizeof(ModConst), hipMemcpyHostToDevice));

    // slot -> spectral position mod t: slot (r, i) is the evaluation at
    // zeta^e, e = (2N-1)^r 3^i mod 2N; the spectral index holding zeta^(2k+1)
    // is brv(k).
    std::vector<uint32_t> pos(N);
    const uint64_t twoN = 2ull * N;
    for (uint32_t r = 0; r < 2; ++r) {
        uint64_t g = r ? twoN - 1 : 1;
        uint64_t p3 = 1;
        for (uint32_t i = 0; i < N / 2; ++i) {
            uint64_t e = (g * p3) % twoN;
            pos[r * (N / 2) + i] = bitrev((uint32_t)((e - 1) / 2), ctx->logN);
            p3 = (p3 * 3) % twoN;
        }
    }
    LOLA_HIP(hipMalloc(&ctx->d_slotpos, N * sizeof(uint32_t)));
    LOLA_HIP(hipMemcpy(ctx->d_slotpos, pos.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice));
    return LOLA_OK;
}

static void pair(uint32_t w, uint32_t q, uint32_t &a, uint32_t &b) {
    a = w % q;
    b = shoup_companion(a, q);
}

static int build_mrc(lola_ctx *ctx) {
    MrcConst &m = ctx->mrc_host;
    memset(&m, 0, sizeof m);
    const uint32_t L = ctx->L, nB = ctx->nB, t = ctx->t;
    m.L = L; m.nB = nB; m.t = t; m.K = ctx->K;
    std::vector<uint64_t> q(L), b(nB);
    for (uint32_t i = 0; i < L; ++i) q[i] = ctx->primes[i];
    for (uint32_t j = 0; j < nB; ++j) b[j] = ctx->primes[ctx->idxB(j)];
    for (uint32_t i = 0; i < L; ++i)
        for (uint32_t k = 0; k < i; ++k) pair((uint32_t)invmod_host(q[k] % q[i], q[i]), (uint32_t)q[i], m.invQ[i][k], m.invQp[i][k]);
    for (uint32_t j = 0; j < nB; ++j) {
        uint64_t w = 1;
        for (uint32_t k = 0; k < L; ++k) {
            pair((uint32_t)w, (uint32_t)b[j], m.wQb[j][k], m.wQbp[j][k]);
            w = mulmod_host(w, q[k], b[j]);
        }
        // w = Q mod b_j now
        pair((uint32_t)w, (uint32_t)b[j], m.Qb[j], m.Qbp[j]);
        pair((uint32_t)invmod_host(w, b[j]), (uint32_t)b[j], m.Qinvb[j], m.Qinvbp[j]);
        pair(t % (uint32_t)b[j], (uint32_t)b[j], m.tb[j], m.tbp[j]);
    }
    {
        uint64_t w = 1;
        for (uint32_t k = 0; k < L; ++k) {
            pair((uint32_t)w, t, m.wQt[k], m.wQtp[k]);
            w = mulmod_host(w, q[k], t);
        }
        pair((uint32_t)invmod_host(w, t), t, m.Qinvt, m.Qinvtp);
        uint64_t Qmodt = w;
        for (uint32_t i = 0; i < L; ++i) {
            // floor(Q/t) = (Q - (Q mod t)) / t = -(Q mod t) t^-1  (mod q_i)
            uint64_t d = mulmod_host((q[i] - Qmodt % q[i]) % q[i], invmod_host(t % q[i], q[i]), q[i]);
            pair((uint32_t)d, (uint32_t)q[i], m.deltaq[i], m.deltaqp[i]);
            pair(t % (uint32_t)q[i], (uint32_t)q[i], m.tq[i], m.tqp[i]);
        }
    }
    {
        std::vector<uint64_t> hr(L);
        for (uint32_t i = 0; i < L; ++i) hr[i] = (q[i] - 1) / 2;  // (Q-1)/2 mod q_i
        std::vector<uint64_t> hd = mrc_host(hr, q);
        for (uint32_t i = 0; i < L; ++i) m.hQ[i] = (uint32_t)hd[i];
    }
    for (uint32_t j = 0; j < nB; ++j)
        for (uint32_t k = 0; k < j; ++k) pair((uint32_t)invmod_host(b[k] % b[j], b[j]), (uint32_t)b[j], m.invB[j][k], m.invBp[j][k]);
    for (uint32_t i = 0; i < L; ++i) {
        uint64_t w = 1;
        for (uint32_t k = 0; k < nB; ++k) {
            pair((uint32_t)w, (uint32_t)q[i], m.wBq[i][k], m.wBqp[i][k]);
            w = mulmod_host(w, b[k], q[i]);
        }
        m.Bq[i] = (uint32_t)w;
    }
    {
        std::vector<uint64_t> hr(nB);
        for (uint32_t j = 0; j < nB; ++j) hr[j] = (b[j] - 1) / 2;
        std::vector<uint64_t> hd = mrc_host(hr, b);
        for (uint32_t j = 0; j < nB; ++j) m.hB[j] = (uint32_t)hd[j];
    }
    const uint32_t K = ctx->K;
    for (uint32_t i = 0; i < L; ++i) {
        uint64_t P = 1;   // the special primes' product mod q_i
        for (uint32_t k = 0; k < K; ++k) P = mulmod_host(P, ctx->primes[L + k] % q[i], q[i]);
        pair((uint32_t)P, (uint32_t)q[i], m.Pq[i], m.Pqp[i]);
        pair((uint32_t)invmod_host(P, q[i]), (uint32_t)q[i], m.Pinvq[i], m.Pinvqp[i]);
    }
    if (K == 2) {
        const uint64_t p0 = ctx->primes[L], p1 = ctx->primes[L + 1];
        m.sp1 = (uint32_t)p1;
        pair((uint32_t)invmod_host(p0 % p1, p1), (uint32_t)p1, m.sp_inv, m.sp_invp);
        m.sp_half0 = (uint32_t)((p0 - 1) / 2);
        m.sp_half1 = (uint32_t)((p1 - 1) / 2);
        for (uint32_t i = 0; i < L; ++i) pair((uint32_t)(p0 % q[i]), (uint32_t)q[i], m.p0q[i], m.p0qp[i]);
        for (uint32_t d = 0; 2 * d + 1 < L; ++d) {
            const uint64_t qa = q[2 * d], qb = q[2 * d + 1];
            m.gqb[d] = (uint32_t)qb;
            pair((uint32_t)invmod_host(qa % qb, qb), (uint32_t)qb, m.ginv[d], m.ginvp[d]);
            for (uint32_t j = 0; j < L + K; ++j) {
                const uint64_t mj = ctx->primes[j];
                pair((uint32_t)(qa % mj), (uint32_t)mj, m.gq[d][j], m.gqp[d][j]);
            }
        }
    }
    LOLA_HIP(hipMalloc(&ctx->d_mrc, sizeof(MrcConst)));
    LOLA_HIP(hipMemcpy(ctx->d_mrc, &m, sizeof(MrcConst), hipMemcpyHostToDevice));
    return LOLA_OK;
}

}  // namespace lola

using namespace lola;

extern "C" {

const char *lola_last_error(void) { return g_last_error.c_str(); }

const char *lola_strerror(int code) {
    switch (code) {
        case LOLA_OK: return "ok";
        case LOLA_E_INVAL: return "invalid argument";
        case LOLA_E_PARAMS: return "invalid parameters";
        case LOLA_E_INSECURE: return "parameters exceed the 128-bit security cap";
        case LOLA_E_SHAPE: return "shape mismatch";
        case LOLA_E_NOKEY: return "missing key";
        case LOLA_E_NOMEM: return "out of device memory";
        case LOLA_E_DEVICE: return "HIP runtime error";
        case LOLA_E_UNSUPPORTED: return "unsupported";
        default: return "unknown error";
    }
}

uint32_t lola_galois_element(uint32_t N, int32_t step) {
    if (N < 8 || (N & (N - 1))) return 0;
    const uint64_t twoN = 2ull * N;
    if (step == LOLA_ROW_SWAP) return (uint32_t)(twoN - 1);
    int64_t k = step % (int64_t)(N / 2);
    if (k < 0) k += N / 2;
    return (uint32_t)powmod_host(3, (uint64_t)k, twoN);
}

int lola_ctx_create(const lola_params *p, int device, lola_ctx **out) {
    if (!p || !out || !p->q) return set_error(LOLA_E_INVAL, "null argument");
    *out = nullptr;
    const uint32_t N = p->N;
    if (N < 1024 || N > 16384 || (N & (N - 1)))
        return set_error(LOLA_E_PARAMS, "N must be a power of two in [1024, 16384]");
    if (p->L < 1 || p->L > (uint32_t)MAXL) return set_error(LOLA_E_PARAMS, "L must be in [1, 12]");
    const uint64_t twoN = 2ull * N;
    std::vector<uint32_t> mods(p->q, p->q + p->L);
    mods.push_back(p->P);
    if (p->P2) mods.push_back(p->P2);
    for (uint32_t m : mods) {
        if (m >= (1u << 30) || !is_prime_u32(m) || (m - 1) % twoN)
            return set_error(LOLA_E_PARAMS, "modulus " + std::to_string(m) + " is not a prime < 2^30 with m = 1 mod 2N");
        // the two-prime digit and special-prime conversions reduce a residue
        // of one such modulus mod another with one conditional subtraction
        if (p->P2 && m < (1u << 29))
            return set_error(LOLA_E_PARAMS, "with a second special prime every modulus must exceed 2^29");
    }
    for (size_t i = 0; i < mods.size(); ++i)
        for (size_t k = 0; k < i; ++k)
            if (mods[i] == mods[k]) return set_error(LOLA_E_PARAMS, "moduli must be distinct");
    if (p->t >= (1u << 26) || !is_prime_u32(p->t) || (p->t - 1) % twoN)
        return set_error(LOLA_E_PARAMS, "t must be a prime < 2^26 with t = 1 mod 2N");
    for (uint32_t m : mods)
        if (m == p->t) return set_error(LOLA_E_PARAMS, "t must be coprime to Q P");
    double bits = 0;
    for (uint32_t m : mods) bits += log2((double)m);
    if (!p->allow_insecure && bits > cap_log2(N))
        return set_error(LOLA_E_INSECURE, "log2(QP) = " + std::to_string(bits) + " exceeds the cap " +
                                              std::to_string(cap_log2(N)) + " for N = " + std::to_string(N));
    int ndev = 0;
    LOLA_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return set_error(LOLA_E_INVAL, "bad device ordinal");
    LOLA_HIP(hipSetDevice(device));

    lola_ctx *ctx = new lola_ctx();
    ctx->device = device;
    ctx->N = N;
    ctx->logN = 0;
    while ((1u << ctx->logN) < N) ++ctx->logN;
    ctx->L = p->L;
    ctx->K = p->P2 ? 2u : 1u;
    ctx->t = p->t;
    ctx->primes = mods;
    // auxiliary basis: primes b = 1 mod 2N below 2^30, outside Q, P and t,
    // until log2(B) >= log2(Q) + log2(t) + log2(N) + 2 (room for the exact
    // product's rounded result, |round(t d / Q)| <= t N Q / 2 + 1).
    double need = log2((double)p->t) + log2((double)N) + 2;
    for (uint32_t i = 0; i < p->L; ++i) need += log2((double)p->q[i]);
    double have = 0;
    uint64_t k = ((1ull << 30) - 1) / twoN;
    std::vector<uint32_t> aux;
    while (have < need && k > 0) {
        uint64_t b = k * twoN + 1;
        --k;
        if (!is_prime_u32(b)) continue;
        if (std::find(mods.begin(), mods.end(), (uint32_t)b) != mods.end() || b == p->t) continue;
        aux.push_back((uint32_t)b);
        have += log2((double)b);
    }
    if (have < need || aux.size() > (size_t)MAXB) {
        delete ctx;
        return set_error(LOLA_E_PARAMS, "cannot build the auxiliary basis");
    }
    ctx->nB = (uint32_t)aux.size();
    for (uint32_t b : aux) ctx->primes.push_back(b);
    ctx->primes.push_back(p->t);
    int rc = build_tables(ctx);
    if (rc == LOLA_OK) rc = build_mrc(ctx);
    if (rc == LOLA_OK) rc = noalloc_setup(device);   // the device's fixed key-switch scratch (lola_rotate_noalloc)
    if (rc != LOLA_OK) {
        lola_ctx_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return LOLA_OK;
}

void lola_ctx_destroy(lola_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (void *p : {(void *)ctx->d_mc, (void *)ctx->d_mrc, (void *)ctx->d_tw,
                    (void *)ctx->d_itw, (void *)ctx->d_slotpos, ctx->d_scratch,
                    (void *)ctx->d_ring})
        if (p) (void)hipFree(p);
    if (ctx->h_ring) (void)hipHostFree(ctx->h_ring);
    for (const lola::TimedLaunch &t : ctx->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t e : ctx->timing_pool) (void)hipEventDestroy(e);
    for (int i = 0; i < lola_ctx::RING_SLABS; ++i)
        if (ctx->ring_ev[i]) (void)hipEventDestroy(ctx->ring_ev[i]);
    delete ctx;
}

int lola_ctx_info(const lola_ctx *ctx, lola_info *info) {
    if (!ctx || !info) return set_error(LOLA_E_INVAL, "null argument");
    info->N = ctx->N;
    info->L = ctx->L;
    info->t = ctx->t;
    info->n_aux = ctx->nB;
    info->poly_words = (uint64_t)ctx->L * ctx->N;
    info->ct_words = 2 * info->poly_words;
    info->sk_words = (uint64_t)(ctx->L + ctx->K) * ctx->N;
    info->ksk_words = (uint64_t)ctx->dnum() * 2 * (ctx->L + ctx->K) * ctx->N;
    info->K = ctx->K;
    info->dnum = ctx->dnum();
    info->scratch_bytes = ctx->scratch_bytes;
    return LOLA_OK;
}

}  // extern "C"
