// Plan executor: loads a plan's constants on the device, binds requests to a
// launch program (one batched launch per op kind per wave, over all
// requests), runs it, or replays it through a captured HIP graph.
#include <cstddef>
#include <cstring>

#include "plan.hpp"

namespace lola {
namespace {

constexpr uint32_t EXEC_KS_CHUNK = 256;
constexpr uint32_t EXEC_MUL_CHUNK = 16;

// Descriptor fields that hold blob-relative offsets until the device blob's
// address is known.
struct Relocs {
    std::vector<size_t> pos;   // byte positions of 64-bit fields inside the blob
};

size_t put_ptrs(Program &prog, Relocs &rel, const std::vector<uint64_t> &v) {
    return prog.put(v);
}

int release_graph(lola_plan *p) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->graph_valid = false;
    return LOLA_OK;
}

int ensure_ws(lola_ctx *ctx, lola_plan *p, size_t words) {
    if (words <= p->ws_words) return LOLA_OK;
    if (p->d_ws) {
        LOLA_HIP(hipDeviceSynchronize());
        LOLA_HIP(hipFree(p->d_ws));
        p->d_ws = nullptr;
        p->ws_words = 0;
    }
    if (hipMalloc(&p->d_ws, words * 4) != hipSuccess)
        return set_error(LOLA_E_NOMEM, "plan workspace allocation of " + std::to_string(words * 4) + " bytes failed");
    p->ws_words = words;
    (void)ctx;
    return LOLA_OK;
}

int ensure_blob(lola_plan *p, size_t bytes) {
    if (bytes <= p->blob_cap) return LOLA_OK;
    if (p->d_blob) {
        LOLA_HIP(hipDeviceSynchronize());
        LOLA_HIP(hipFree(p->d_blob));
        LOLA_HIP(hipHostFree(p->h_blob));
        p->d_blob = p->h_blob = nullptr;
    }
    size_t cap = bytes + bytes / 4 + 4096;
    if (hipMalloc((void **)&p->d_blob, cap) != hipSuccess) return set_error(LOLA_E_NOMEM, "plan blob allocation failed");
    LOLA_HIP(hipHostMalloc((void **)&p->h_blob, cap, hipHostMallocDefault));
    p->blob_cap = cap;
    return LOLA_OK;
}

std::vector<std::vector<const uint32_t *>> request_ptrs(const lola_plan *p, const lola_request *reqs, uint32_t n) {
    std::vector<std::vector<const uint32_t *>> v(n);
    for (uint32_t r = 0; r < n; ++r) {
        v[r].push_back(reqs[r].rlk_dev);
        for (size_t g = 0; g < p->galois.size(); ++g) v[r].push_back(reqs[r].gk_dev[g]);
        for (uint32_t i = 0; i < p->n_inputs; ++i) v[r].push_back(reqs[r].in_dev[i]);
        for (size_t o = 0; o < p->outputs.size(); ++o) v[r].push_back(reqs[r].out_dev[o]);
    }
    return v;
}

int validate(const lola_ctx *ctx, const lola_plan *p, const lola_request *reqs, uint32_t n) {
    if (p->loaded_for != ctx) return set_error(LOLA_E_INVAL, "plan constants not loaded for this context (lola_plan_load)");
    for (uint32_t r = 0; r < n; ++r) {
        if (!reqs[r].in_dev || !reqs[r].out_dev || (!p->galois.empty() && !reqs[r].gk_dev))
            return set_error(LOLA_E_INVAL, "request arrays missing");
        bool sq = false;
        for (const Op &o : p->ops) sq |= o.kind == OP_SQUARE;
        if (sq && !reqs[r].rlk_dev) return set_error(LOLA_E_NOKEY, "plan squares but the request has no relinearisation key");
        for (size_t g = 0; g < p->galois.size(); ++g)
            if (!reqs[r].gk_dev[g]) return set_error(LOLA_E_NOKEY, "missing Galois key " + std::to_string(p->galois[g]));
        for (uint32_t i = 0; i < p->n_inputs; ++i)
            if (!reqs[r].in_dev[i]) return set_error(LOLA_E_INVAL, "null input ciphertext");
        for (size_t o = 0; o < p->outputs.size(); ++o) {
            if (!reqs[r].out_dev[o]) return set_error(LOLA_E_INVAL, "null output ciphertext");
            for (uint32_t i = 0; i < p->n_inputs; ++i)
                if (reqs[r].out_dev[o] == reqs[r].in_dev[i]) return set_error(LOLA_E_INVAL, "output aliases an input");
        }
    }
    return LOLA_OK;
}

// Builds the launch program for n requests.  Pointers into the blob itself
// (lincomb source lists and scalar tables) are recorded as offsets and
// relocated by the caller.
int bind(lola_ctx *ctx, lola_plan *p, const lola_request *reqs, uint32_t n, Relocs &rel) {
    const size_t N = p->N, L = p->L, CT = 2 * L * N, CT3 = 3 * L * N;
    // workspace: registers, square temporaries, scratch
    size_t max_ks = 0;
    std::vector<size_t> ks_per_wave(p->n_waves + 1, 0);
    for (const Op &o : p->ops)
        if (o.kind == OP_ROTADD || o.kind == OP_ROT || o.kind == OP_SQUARE) ks_per_wave[o.level] += n;
    for (size_t c : ks_per_wave) max_ks = std::max(max_ks, c);
    const uint32_t ks_chunk = (uint32_t)std::max<size_t>(1, std::min<size_t>(EXEC_KS_CHUNK, max_ks));
    const uint32_t mul_chunk = (uint32_t)std::max<size_t>(1, std::min<size_t>(EXEC_MUL_CHUNK, (size_t)p->max_squares_per_wave * n));
    const size_t scratch_words = std::max(ks_chunk * ks_scratch_words(ctx), mul_chunk * mul_scratch_words(ctx));
    const size_t reg_words = (size_t)n * p->n_phys * CT;
    const size_t sq_words = (size_t)n * std::max<uint32_t>(p->max_squares_per_wave, 1) * CT3;
    int rc = ensure_ws(ctx, p, reg_words + sq_words + scratch_words);
    if (rc) return rc;
    uint32_t *regs = p->d_ws, *sqt = p->d_ws + reg_words, *scratch = p->d_ws + reg_words + sq_words;
    auto ptr = [&](uint32_t r, int v) -> uint32_t * {
        if (v < (int)p->n_inputs) return const_cast<uint32_t *>(reqs[r].in_dev[v]);
        if (p->phys[v] < 0) {
            for (size_t o = 0; o < p->outputs.size(); ++o)
                if (p->outputs[o] == v) return reqs[r].out_dev[o];
            return nullptr;
        }
        return regs + ((size_t)r * p->n_phys + p->phys[v]) * CT;
    };
    auto gk = [&](uint32_t r, uint32_t g) -> const uint32_t * {
        size_t k = std::lower_bound(p->galois.begin(), p->galois.end(), g) - p->galois.begin();
        return reqs[r].gk_dev[k];
    };
    Program &prog = p->prog;
    prog = Program();
    // lincomb scalar tables, one per op: [n_src][2][L]
    std::vector<size_t> wtab(p->ops.size(), 0);
    for (size_t i = 0; i < p->ops.size(); ++i) {
        const Op &o = p->ops[i];
        if (o.kind != OP_LINCOMB) continue;
        std::vector<uint32_t> tab(o.srcs.size() * 2 * L);
        for (size_t k = 0; k < o.srcs.size(); ++k) {
            int64_t w = o.w[k] % (int64_t)p->t;
            if (w < 0) w += p->t;
            if (w > (int64_t)(p->t / 2)) w -= p->t;   // [w]_t
            for (size_t j = 0; j < L; ++j) {
                const int64_t q = ctx->primes[j];
                int64_t r = w % q;
                if (r < 0) r += q;
                tab[(2 * k) * L + j] = (uint32_t)r;
                tab[(2 * k + 1) * L + j] = shoup_companion((uint32_t)r, (uint32_t)q);
            }
        }
        wtab[i] = prog.put(tab);
    }
    for (uint32_t lev = 1; lev <= p->n_waves; ++lev) {
        std::vector<LinJob> lin;
        std::vector<size_t> lin_lists;
        std::vector<PlainJob> plain;
        std::vector<KsJob> ks, relin;
        std::vector<MulJob> muls;
        uint32_t sq_slot = 0;
        for (uint32_t r = 0; r < n; ++r) {
            sq_slot = 0;
            for (size_t i = 0; i < p->ops.size(); ++i) {
                const Op &o = p->ops[i];
                if ((uint32_t)o.level != lev) continue;
                uint32_t *dst = ptr(r, o.dst);
                switch (o.kind) {
                    case OP_LINCOMB: {
                        std::vector<uint64_t> lst;
                        for (int s : o.srcs) lst.push_back((uint64_t)(uintptr_t)ptr(r, s));
                        const size_t off = put_ptrs(prog, rel, lst);
                        LinJob j{};
                        j.srcs = (const uint32_t *const *)(uintptr_t)off;        // relocated
                        j.w = (const uint32_t *)(uintptr_t)wtab[i];              // relocated
                        j.add = o.cadd >= 0 ? p->d_cadd[o.cadd] : nullptr;
                        j.dst = dst;
                        j.n_src = (uint32_t)o.srcs.size();
                        lin.push_back(j);
                        break;
                    }
                    case OP_MULPLAIN:
                        plain.push_back(PlainJob{ptr(r, o.src), p->d_cmul[o.cmul],
                                                 o.cadd >= 0 ? p->d_cadd[o.cadd] : nullptr, dst});
                        break;
                    case OP_ADDPLAIN:
                        plain.push_back(PlainJob{ptr(r, o.src), nullptr, p->d_cadd[o.cadd], dst});
                        break;
                    case OP_ROTADD:
                    case OP_ROT: {
                        const uint32_t *src = ptr(r, o.src);
                        KsJob j{};
                        j.x = src + L * N;
                        j.key = gk(r, o.galois);
                        j.add0 = src;
                        j.addct = o.kind == OP_ROTADD ? ptr(r, o.addend) : nullptr;
                        j.out = dst;
                        j.galois = o.galois;
                        ks.push_back(j);
                        break;
                    }
                    case OP_SQUARE: {
                        const uint32_t *src = ptr(r, o.src);
                        uint32_t *t3 = sqt + ((size_t)r * std::max<uint32_t>(p->max_squares_per_wave, 1) + sq_slot++) * CT3;
                        muls.push_back(MulJob{src, src, t3, nullptr});
                        KsJob j{};
                        j.x = t3 + 2 * L * N;
                        j.key = reqs[r].rlk_dev;
                        j.add0 = t3;
                        j.add1 = t3 + L * N;
                        j.out = dst;
                        relin.push_back(j);
                        break;
                    }
                }
            }
        }
        if (!lin.empty()) {
            const size_t off = prog.put(lin);
            for (size_t k = 0; k < lin.size(); ++k) {
                rel.pos.push_back(off + k * sizeof(LinJob) + offsetof(LinJob, srcs));
                rel.pos.push_back(off + k * sizeof(LinJob) + offsetof(LinJob, w));
            }
            prog.launches.push_back(Launch{LK_LIN, (uint32_t)lin.size(), off});
        }
        prog.launch(LK_PLAIN, plain);
        if (!muls.empty()) {
            program_mul(ctx, prog, muls, scratch, mul_chunk);
            program_keyswitch(ctx, prog, relin, scratch, ks_chunk);
        }
        program_keyswitch(ctx, prog, ks, scratch, ks_chunk);
    }
    return LOLA_OK;
}

int upload(lola_plan *p, const Relocs &rel, hipStream_t s) {
    Program &prog = p->prog;
    int rc = ensure_blob(p, prog.blob.size());
    if (rc) return rc;
    // the previous upload from h_blob must be complete before rewriting it
    LOLA_HIP(hipStreamSynchronize(s));
    memcpy(p->h_blob, prog.blob.data(), prog.blob.size());
    for (size_t pos : rel.pos) {
        uint64_t v;
        memcpy(&v, p->h_blob + pos, 8);
        v += (uint64_t)(uintptr_t)p->d_blob;
        memcpy(p->h_blob + pos, &v, 8);
    }
    LOLA_HIP(hipMemcpyAsync(p->d_blob, p->h_blob, prog.blob.size(), hipMemcpyHostToDevice, s));
    return LOLA_OK;
}

int prepare(lola_ctx *ctx, lola_plan *p, const lola_request *reqs, uint32_t n, hipStream_t s, bool *rebound) {
    int rc = validate(ctx, p, reqs, n);
    if (rc) return rc;
    auto ptrs = request_ptrs(p, reqs, n);
    *rebound = false;
    if (p->prog_valid && ptrs == p->bound_ptrs) return LOLA_OK;
    Relocs rel;
    p->prog_valid = false;
    release_graph(p);
    if ((rc = bind(ctx, p, reqs, n, rel))) return rc;
    if ((rc = upload(p, rel, s))) return rc;
    p->bound_ptrs = ptrs;
    p->prog_valid = true;
    *rebound = true;
    return LOLA_OK;
}

}  // namespace
}  // namespace lola

using namespace lola;

extern "C" {

int lola_plan_load(lola_ctx *ctx, lola_plan *p, lola_stream stream) {
    if (!ctx || !p) return set_error(LOLA_E_INVAL, "null argument");
    if (p->N != ctx->N || p->L != ctx->L || p->t != ctx->t) return set_error(LOLA_E_SHAPE, "plan compiled for other parameters");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = ctx->N, L = ctx->L;
    for (uint32_t *q : p->d_cmul) if (q) (void)hipFree(q);
    for (uint32_t *q : p->d_cadd) if (q) (void)hipFree(q);
    p->d_cmul.assign(p->consts.size(), nullptr);
    p->d_cadd.assign(p->consts.size(), nullptr);
    int64_t *d_slots = nullptr;
    uint32_t *d_pt = nullptr;
    LOLA_HIP(hipMalloc(&d_slots, N * 8));
    LOLA_HIP(hipMalloc(&d_pt, N * 4));
    int rc = LOLA_OK;
    for (size_t c = 0; c < p->consts.size() && !rc; ++c) {
        LOLA_HIP(hipMemcpyAsync(d_slots, p->consts[c].data(), N * 8, hipMemcpyHostToDevice, s));
        rc = lola_encode(ctx, d_slots, d_pt, stream);
        if (!rc && p->const_mul[c]) {
            if (hipMalloc(&p->d_cmul[c], L * N * 4) != hipSuccess) rc = set_error(LOLA_E_NOMEM, "constant allocation");
            else rc = lola_plain_mul_form(ctx, d_pt, p->d_cmul[c], stream);
        }
        if (!rc && p->const_add[c]) {
            if (hipMalloc(&p->d_cadd[c], L * N * 4) != hipSuccess) rc = set_error(LOLA_E_NOMEM, "constant allocation");
            else rc = lola_plain_add_form(ctx, d_pt, p->d_cadd[c], stream);
        }
        // the slot staging buffer is reused: wait for this constant's upload
        if (!rc) LOLA_HIP(hipStreamSynchronize(s));
    }
    (void)hipFree(d_slots);
    (void)hipFree(d_pt);
    if (rc) return rc;
    p->loaded_for = ctx;
    p->prog_valid = false;
    release_graph(p);
    return LOLA_OK;
}

void lola_plan_destroy(lola_plan *p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    release_graph(p);
    for (uint32_t *q : p->d_cmul) if (q) (void)hipFree(q);
    for (uint32_t *q : p->d_cadd) if (q) (void)hipFree(q);
    if (p->d_ws) (void)hipFree(p->d_ws);
    if (p->d_blob) (void)hipFree(p->d_blob);
    if (p->h_blob) (void)hipHostFree(p->h_blob);
    delete p;
}

int lola_evaluate(lola_ctx *ctx, lola_plan *p, const lola_request *reqs, uint32_t n, lola_stream stream) {
    if (!ctx || !p || (!reqs && n)) return set_error(LOLA_E_INVAL, "null argument");
    if (n == 0) return LOLA_OK;
    hipStream_t s = (hipStream_t)stream;
    bool rebound = false;
    int rc = prepare(ctx, p, reqs, n, s, &rebound);
    if (rc) return rc;
    return program_run(ctx, p->prog, p->d_blob, s);
}

int lola_evaluate_graph(lola_ctx *ctx, lola_plan *p, const lola_request *reqs, uint32_t n, lola_stream stream) {
    if (!ctx || !p || (!reqs && n)) return set_error(LOLA_E_INVAL, "null argument");
    if (n == 0) return LOLA_OK;
    if (ctx->timing) return set_error(LOLA_E_INVAL, "kernel timing and graph replay are exclusive");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return set_error(LOLA_E_INVAL, "graph replay needs a non-default stream");
    bool rebound = false;
    int rc = prepare(ctx, p, reqs, n, s, &rebound);
    if (rc) return rc;
    if (!p->graph_valid) {
        LOLA_HIP(hipStreamSynchronize(s));   // blob upload done before capture
        LOLA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        rc = program_run(ctx, p->prog, p->d_blob, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return check_hip(e, "hipStreamEndCapture");
        p->graph = g;
        LOLA_HIP(hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0));
        p->graph_valid = true;
    }
    LOLA_HIP(hipGraphLaunch(p->graph_exec, s));
    return LOLA_OK;
}

}  // extern "C"
