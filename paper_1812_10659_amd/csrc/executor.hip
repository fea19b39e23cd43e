// Plan executor: loads a plan's constants on the device, emits the jobs of
// each wave for any set of requests (one batched launch per op kind per wave,
// over all requests), runs a bound program, or replays it through a captured
// HIP graph.  The serving loop reuses emit_level / program_level.
#include <algorithm>
#include <cstddef>
#include <cstring>

#include "plan.hpp"

namespace lola {

constexpr uint32_t EXEC_KS_CHUNK = 256;
constexpr uint32_t EXEC_MUL_CHUNK = 16;
constexpr uint32_t EXEC_LANE_MIN_REQUESTS = 16;   // batches from this size run as two lanes

int validate_request(const lola_plan *p, const lola_request &r) {
    if (!r.in_dev || !r.out_dev || (!p->galois.empty() && !r.gk_dev))
        return set_error(LOLA_E_INVAL, "request arrays missing");
    if (p->max_squares_per_wave > 0 && !r.rlk_dev)
        return set_error(LOLA_E_NOKEY, "plan squares but the request has no relinearisation key");
    for (size_t g = 0; g < p->galois.size(); ++g)
        if (!r.gk_dev[g]) return set_error(LOLA_E_NOKEY, "missing Galois key " + std::to_string(p->galois[g]));
    for (uint32_t i = 0; i < p->n_inputs; ++i)
        if (!r.in_dev[i]) return set_error(LOLA_E_INVAL, "null input ciphertext");
    for (size_t o = 0; o < p->outputs.size(); ++o) {
        if (!r.out_dev[o]) return set_error(LOLA_E_INVAL, "null output ciphertext");
        for (uint32_t i = 0; i < p->n_inputs; ++i)
            if (r.out_dev[o] == r.in_dev[i]) return set_error(LOLA_E_INVAL, "output aliases an input");
    }
    return LOLA_OK;
}

int emit_level(const lola_ctx *ctx, const lola_plan *p, const ReqView &rv, uint32_t level, LevelJobs &out) {
    const size_t N = p->N, L = p->L, CT = 2 * L * N, CT3 = 3 * L * N;
    const lola_request &rq = *rv.req;
    auto ptr = [&](int v) -> uint32_t * {
        if (v < (int)p->n_inputs) return const_cast<uint32_t *>(rq.in_dev[v]);
        if (p->phys[v] < 0) {
            for (size_t o = 0; o < p->outputs.size(); ++o)
                if (p->outputs[o] == v) return rq.out_dev[o];
            return nullptr;
        }
        return rv.regs + (size_t)p->phys[v] * CT;
    };
    auto gk = [&](uint32_t g) -> const uint32_t * {
        size_t k = std::lower_bound(p->galois.begin(), p->galois.end(), g) - p->galois.begin();
        return rq.gk_dev[k];
    };
    uint32_t sq_slot = 0;
    std::vector<const uint32_t *> hoisted;   // sources of hoisted rotations in this wave
    const size_t HW = ks_hoist_words(ctx);
    for (int i : p->level_ops[level]) {
        const Op &o = p->ops[i];
        uint32_t *dst = ptr(o.dst);
        if (!dst) return set_error(LOLA_E_INVAL, "internal: unassigned register");
        switch (o.kind) {
            case OP_LINCOMB: {
                LinJob j{};
                for (size_t k = 0; k < o.srcs.size(); ++k) j.srcs[k] = ptr(o.srcs[k]);
                j.w[0] = p->d_wtab[i];
                j.add[0] = o.cadd >= 0 ? p->d_cadd[o.cadd] : nullptr;
                j.dst[0] = dst;
                j.n_src = (uint32_t)o.srcs.size();
                j.n_dst = 1;
                out.lin.push_back(j);
                break;
            }
            case OP_MULPLAIN:
                out.plain.push_back(PlainJob{ptr(o.src), p->d_cmul[o.cmul], o.cadd >= 0 ? p->d_cadd[o.cadd] : nullptr, dst});
                break;
            case OP_ADDPLAIN:
                out.plain.push_back(PlainJob{ptr(o.src), nullptr, p->d_cadd[o.cadd], dst});
                break;
            case OP_ROTADD:
            case OP_ROT: {
                const uint32_t *src = ptr(o.src);
                if (o.kind == OP_ROT && o.hoist) {
                    size_t k = std::find(hoisted.begin(), hoisted.end(), src) - hoisted.begin();
                    if (k == hoisted.size()) {
                        if (k >= p->max_hoist_per_wave) return set_error(LOLA_E_INVAL, "internal: hoist areas");
                        hoisted.push_back(src);
                        KsJob hs{};
                        hs.x = src + L * N;
                        hs.scratch = rv.hoist + k * HW;
                        hs.galois = 1;
                        out.hsrc.push_back(hs);
                    }
                    KsJob j{};
                    j.x = src + L * N;
                    j.key = gk(o.galois);
                    j.add0 = src;
                    j.out = dst;
                    j.galois = o.galois;
                    j.hoist = rv.hoist + k * HW;
                    out.hrot.push_back(j);
                    break;
                }
                KsJob j{};
                j.x = src + L * N;
                j.key = gk(o.galois);
                j.add0 = src;
                j.addct = o.kind == OP_ROTADD ? ptr(o.addend) : nullptr;
                j.out = dst;
                j.galois = o.galois;
                out.ks.push_back(j);
                break;
            }
            case OP_SQUARE: {
                const uint32_t *src = ptr(o.src);
                uint32_t *t3 = rv.sq + (size_t)(sq_slot++) * CT3;
                out.muls.push_back(MulJob{src, src, t3, nullptr});
                KsJob j{};
                j.x = t3 + 2 * L * N;
                j.key = rq.rlk_dev;
                j.add0 = t3;
                j.add1 = t3 + L * N;
                j.out = dst;
                out.relin.push_back(j);
                break;
            }
        }
    }
    return LOLA_OK;
}

size_t level_scratch_words(const lola_ctx *ctx, uint32_t ks_chunk, uint32_t mul_chunk) {
    return std::max(ks_chunk_words(ctx, ks_chunk), mul_chunk * mul_scratch_words(ctx));
}

void program_level(const lola_ctx *ctx, Program &prog, LevelJobs &jobs, uint32_t *scratch, uint32_t ks_chunk,
                   uint32_t mul_chunk) {
    prog.launch(LK_LIN, group_lincombs(jobs.lin));
    prog.launch(LK_PLAIN, jobs.plain);
    if (!jobs.muls.empty()) {
        program_mul(ctx, prog, jobs.muls, scratch, mul_chunk);
        program_keyswitch(ctx, prog, jobs.relin, scratch, ks_chunk);
    }
    program_keyswitch(ctx, prog, jobs.ks, scratch, ks_chunk);
    if (!jobs.hrot.empty()) {
        // sources first (their hoist areas are their own), then the rotations
        // in chunks over the level scratch
        prog.launch(LK_KS_HSRC, jobs.hsrc);
        program_keyswitch(ctx, prog, jobs.hrot, scratch, ks_chunk, LK_KS_HROT);
    }
}

// Launches two programs, interleaved launch by launch so both streams have
// work queued from the start.
int run_two(lola_ctx *ctx, const Program &a, const uint8_t *da, hipStream_t sa, const Program &b,
            const uint8_t *db, hipStream_t sb) {
    const size_t na = a.launches.size(), nb = b.launches.size();
    size_t i = 0, j = 0;
    while (i < na || j < nb) {
        // keep the two lanes' progress proportional
        const bool take_a = j >= nb || (i < na && i * nb <= j * na);
        int rc = take_a ? program_run_launch(ctx, a.launches[i++], da, sa)
                        : program_run_launch(ctx, b.launches[j++], db, sb);
        if (rc) return rc;
    }
    return LOLA_OK;
}

namespace {

int release_graph(lola_plan *p) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->graph_valid = false;
    return LOLA_OK;
}

int ensure_ws(ExecLane &ln, size_t words) {
    if (words <= ln.ws_words) return LOLA_OK;
    if (ln.d_ws) {
        LOLA_HIP(hipDeviceSynchronize());
        LOLA_HIP(hipFree(ln.d_ws));
        ln.d_ws = nullptr;
        ln.ws_words = 0;
    }
    if (hipMalloc(&ln.d_ws, words * 4) != hipSuccess)
        return set_error(LOLA_E_NOMEM, "plan workspace allocation of " + std::to_string(words * 4) + " bytes failed");
    ln.ws_words = words;
    return LOLA_OK;
}

int ensure_blob(ExecLane &ln, size_t bytes) {
    if (bytes <= ln.blob_cap) return LOLA_OK;
    if (ln.d_blob) {
        LOLA_HIP(hipDeviceSynchronize());
        LOLA_HIP(hipFree(ln.d_blob));
        LOLA_HIP(hipHostFree(ln.h_blob));
        ln.d_blob = ln.h_blob = nullptr;
    }
    size_t cap = bytes + bytes / 4 + 4096;
    if (hipMalloc((void **)&ln.d_blob, cap) != hipSuccess) return set_error(LOLA_E_NOMEM, "plan blob allocation failed");
    LOLA_HIP(hipHostMalloc((void **)&ln.h_blob, cap, hipHostMallocDefault));
    ln.blob_cap = cap;
    return LOLA_OK;
}

void free_lane(ExecLane &ln) {
    if (ln.d_ws) (void)hipFree(ln.d_ws);
    if (ln.d_blob) (void)hipFree(ln.d_blob);
    if (ln.h_blob) (void)hipHostFree(ln.h_blob);
    ln = ExecLane();
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

// Builds the whole launch program for n requests evaluated together.
int bind(lola_ctx *ctx, lola_plan *p, ExecLane &ln, const lola_request *reqs, uint32_t n) {
    const size_t N = p->N, L = p->L, CT = 2 * L * N, CT3 = 3 * L * N;
    size_t max_ks = 1;
    for (uint32_t lev = 1; lev <= p->n_waves; ++lev) {
        size_t c = 0;
        for (int i : p->level_ops[lev]) {
            const int k = p->ops[i].kind;
            c += (k == OP_ROTADD || k == OP_ROT || k == OP_SQUARE) ? n : 0;
        }
        max_ks = std::max(max_ks, c);
    }
    const uint32_t ks_chunk = (uint32_t)std::min<size_t>(EXEC_KS_CHUNK, max_ks);
    const uint32_t mul_chunk =
        (uint32_t)std::max<size_t>(1, std::min<size_t>(EXEC_MUL_CHUNK, (size_t)p->max_squares_per_wave * n));
    const uint32_t nsq = std::max<uint32_t>(p->max_squares_per_wave, 1);
    const size_t reg_words = (size_t)n * p->n_phys * CT;
    const size_t sq_words = (size_t)n * nsq * CT3;
    const size_t hoist_per_req = (size_t)p->max_hoist_per_wave * ks_hoist_words(ctx);
    const size_t hoist_words = (size_t)n * hoist_per_req;
    int rc = ensure_ws(ln, reg_words + sq_words + hoist_words + level_scratch_words(ctx, ks_chunk, mul_chunk));
    if (rc) return rc;
    uint32_t *regs = ln.d_ws, *sqt = ln.d_ws + reg_words, *hst = ln.d_ws + reg_words + sq_words;
    uint32_t *scratch = hst + hoist_words;
    std::vector<ReqView> views(n);
    for (uint32_t r = 0; r < n; ++r)
        views[r] = ReqView{&reqs[r], regs + (size_t)r * p->n_phys * CT, sqt + (size_t)r * nsq * CT3,
                           hst + (size_t)r * hoist_per_req};
    Program &prog = ln.prog;
    prog = Program();
    for (uint32_t lev = 1; lev <= p->n_waves; ++lev) {
        LevelJobs jobs;
        for (uint32_t r = 0; r < n; ++r)
            if ((rc = emit_level(ctx, p, views[r], lev, jobs))) return rc;
        program_level(ctx, prog, jobs, scratch, ks_chunk, mul_chunk);
    }
    return LOLA_OK;
}

int upload(ExecLane &ln, hipStream_t s) {
    Program &prog = ln.prog;
    int rc = ensure_blob(ln, prog.blob.size());
    if (rc) return rc;
    LOLA_HIP(hipStreamSynchronize(s));   // the previous upload from h_blob is complete
    memcpy(ln.h_blob, prog.blob.data(), prog.blob.size());
    LOLA_HIP(hipMemcpyAsync(ln.d_blob, ln.h_blob, prog.blob.size(), hipMemcpyHostToDevice, s));
    return LOLA_OK;
}

// Binds (when the request pointers changed) and uploads the programs of
// n_lanes lanes: lane k takes requests [k * half, ...), half = ceil(n / n_lanes).
int prepare(lola_ctx *ctx, lola_plan *p, const lola_request *reqs, uint32_t n, hipStream_t s, uint32_t n_lanes) {
    if (p->loaded_for != ctx) return set_error(LOLA_E_INVAL, "plan constants not loaded for this context (lola_plan_load)");
    for (uint32_t r = 0; r < n; ++r) {
        int rc = validate_request(p, reqs[r]);
        if (rc) return rc;
    }
    const uint32_t half = (n + n_lanes - 1) / n_lanes;
    for (uint32_t k = 0; k < 2; ++k) {
        ExecLane &ln = p->lanes[k];
        const uint32_t off = std::min(n, k * half), cnt = k < n_lanes ? std::min(half, n - off) : 0;
        auto ptrs = request_ptrs(p, reqs + off, cnt);
        if (ln.prog_valid && ptrs == ln.bound_ptrs) continue;
        ln.prog_valid = false;
        release_graph(p);   // a captured graph runs the lanes' programs
        if (cnt == 0) {   // unused lane: nothing bound
            ln.prog = Program();
            ln.bound_ptrs = ptrs;
            ln.prog_valid = true;
            continue;
        }
        int rc = bind(ctx, p, ln, reqs + off, cnt);
        if (rc) return rc;
        if ((rc = upload(ln, s))) return rc;
        ln.bound_ptrs = ptrs;
        ln.prog_valid = true;
    }
    return LOLA_OK;
}

// The two bound lanes' programs, as above.
int run_two(lola_ctx *ctx, const ExecLane &a, hipStream_t sa, const ExecLane &b, hipStream_t sb) {
    return run_two(ctx, a.prog, a.d_blob, sa, b.prog, b.d_blob, sb);
}

void free_consts(lola_plan *p) {
    for (auto *v : {&p->d_cmul, &p->d_cadd, &p->d_wtab})
        for (uint32_t *q : *v)
            if (q) (void)hipFree(q);
    p->d_cmul.clear();
    p->d_cadd.clear();
    p->d_wtab.clear();
}

}  // namespace
}  // namespace lola

using namespace lola;

extern "C" {

int lola_plan_load(lola_ctx *ctx, lola_plan *p, lola_stream stream) {
    if (!ctx || !p) return set_error(LOLA_E_INVAL, "null argument");
    if (p->N != ctx->N || p->L != ctx->L || p->t != ctx->t || p->K != ctx->K)
        return set_error(LOLA_E_SHAPE, "plan compiled for other parameters");
    hipStream_t s = (hipStream_t)stream;
    const size_t N = ctx->N, L = ctx->L;
    // Everything is built into fresh buffers first.  On any failure they are
    // freed and the plan keeps its previous constants, binding and graph, all
    // still valid; only a complete load replaces them.
    std::vector<uint32_t *> cmul(p->consts.size(), nullptr), cadd(p->consts.size(), nullptr),
        wtab(p->ops.size(), nullptr);
    int64_t *d_slots = nullptr;
    uint32_t *d_pt = nullptr;
    auto release_new = [&]() {
        (void)hipStreamSynchronize(s);   // no queued work may still read them
        for (auto *v : {&cmul, &cadd, &wtab})
            for (uint32_t *q : *v)
                if (q) (void)hipFree(q);
        if (d_slots) (void)hipFree(d_slots);
        if (d_pt) (void)hipFree(d_pt);
    };
    int rc = LOLA_OK;
    if (hipMalloc(&d_slots, N * 8) != hipSuccess || hipMalloc(&d_pt, N * 4) != hipSuccess)
        rc = set_error(LOLA_E_NOMEM, "staging allocation");
    for (size_t c = 0; c < p->consts.size() && !rc; ++c) {
        if (hipMemcpyAsync(d_slots, p->consts[c].data(), N * 8, hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = set_error(LOLA_E_DEVICE, "constant upload");
            break;
        }
        rc = lola_encode(ctx, d_slots, d_pt, stream);
        if (!rc && p->const_mul[c]) {
            if (hipMalloc(&cmul[c], L * N * 4) != hipSuccess) rc = set_error(LOLA_E_NOMEM, "constant allocation");
            else rc = lola_plain_mul_form(ctx, d_pt, cmul[c], stream);
        }
        if (!rc && p->const_add[c]) {
            if (hipMalloc(&cadd[c], L * N * 4) != hipSuccess) rc = set_error(LOLA_E_NOMEM, "constant allocation");
            else rc = lola_plain_add_form(ctx, d_pt, cadd[c], stream);
        }
        // the slot staging buffer is reused: wait for this constant's upload
        if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = set_error(LOLA_E_DEVICE, "constant upload");
    }
    // linear-combination scalars: [w]_t reduced per prime, and in Montgomery
    // form (w 2^32 mod q) for the kernel's 64-bit multiply-add
    for (size_t i = 0; i < p->ops.size() && !rc; ++i) {
        const Op &o = p->ops[i];
        if (o.kind != OP_LINCOMB) continue;
        std::vector<uint32_t> tab(o.srcs.size() * 2 * L);
        for (size_t k = 0; k < o.srcs.size(); ++k) {
            int64_t w = o.w[k] % (int64_t)p->t;
            if (w < 0) w += p->t;
            if (w > (int64_t)(p->t / 2)) w -= p->t;
            for (size_t j = 0; j < L; ++j) {
                const int64_t q = ctx->primes[j];
                int64_t r = w % q;
                if (r < 0) r += q;
                tab[(2 * k) * L + j] = (uint32_t)r;
                tab[(2 * k + 1) * L + j] = (uint32_t)mulmod_host((uint64_t)r, (1ull << 32) % (uint64_t)q, (uint64_t)q);
            }
        }
        if (hipMalloc(&wtab[i], tab.size() * 4) != hipSuccess) rc = set_error(LOLA_E_NOMEM, "table allocation");
        else if (hipMemcpy(wtab[i], tab.data(), tab.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            rc = set_error(LOLA_E_DEVICE, "table upload");
    }
    if (rc) {
        release_new();
        return rc;
    }
    (void)hipFree(d_slots);
    (void)hipFree(d_pt);
    // replace the previous constants: nothing bound or captured may refer to
    // them afterwards (hipFree waits for the device)
    p->lanes[0].prog_valid = p->lanes[1].prog_valid = false;
    release_graph(p);
    free_consts(p);
    p->d_cmul.swap(cmul);
    p->d_cadd.swap(cadd);
    p->d_wtab.swap(wtab);
    p->loaded_for = ctx;
    return LOLA_OK;
}

void lola_plan_destroy(lola_plan *p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    release_graph(p);
    free_consts(p);
    free_lane(p->lanes[0]);
    free_lane(p->lanes[1]);
    if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    if (p->join_ev) (void)hipEventDestroy(p->join_ev);
    delete p;
}

// The second lane's stream (default priority) and its fork/join events.
static int ensure_side(lola_plan *p) {
    if (p->side_stream) return LOLA_OK;
    LOLA_HIP(hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking));
    LOLA_HIP(hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming));
    LOLA_HIP(hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming));
    return LOLA_OK;
}

// Issues the bound lanes' programs: one lane on s, or two forked from s onto
// the plan's side stream and joined back (also while s is being captured:
// the side stream then joins the capture through the fork event, so the
// stream and events must exist before the capture begins).
static int run_lanes(lola_ctx *ctx, lola_plan *p, uint32_t n_lanes, hipStream_t s) {
    if (n_lanes == 1) return program_run(ctx, p->lanes[0].prog, p->lanes[0].d_blob, s);
    int rc = ensure_side(p);
    if (rc) return rc;
    LOLA_HIP(hipEventRecord(p->fork_ev, s));   // inputs and uploads on s come first
    LOLA_HIP(hipStreamWaitEvent(p->side_stream, p->fork_ev, 0));
    rc = run_two(ctx, p->lanes[0], s, p->lanes[1], p->side_stream);
    // join even after an error, so s never runs ahead of queued side work
    LOLA_HIP(hipEventRecord(p->join_ev, p->side_stream));
    LOLA_HIP(hipStreamWaitEvent(s, p->join_ev, 0));
    return rc;
}

int lola_evaluate(lola_ctx *ctx, lola_plan *p, const lola_request *reqs, uint32_t n, lola_stream stream) {
    if (!ctx || !p || (!reqs && n)) return set_error(LOLA_E_INVAL, "null argument");
    if (n == 0) return LOLA_OK;
    hipStream_t s = (hipStream_t)stream;
    // two lanes for batches large enough that each half still fills the
    // launches: kernels of one half run in the other's launch tails.  Kernel
    // timing measures launches alone, so it keeps one lane.
    const uint32_t n_lanes = (!ctx->timing && n >= EXEC_LANE_MIN_REQUESTS && p->max_lanes >= 2) ? 2 : 1;
    int rc = prepare(ctx, p, reqs, n, s, n_lanes);
    if (rc) return rc;
    return run_lanes(ctx, p, n_lanes, s);
}

int lola_plan_set_lanes(lola_plan *p, uint32_t max_lanes) {
    if (!p) return set_error(LOLA_E_INVAL, "null argument");
    if (max_lanes < 1 || max_lanes > 2) return set_error(LOLA_E_INVAL, "lanes must be 1 or 2");
    p->max_lanes = max_lanes;
    return LOLA_OK;
}

int lola_evaluate_graph(lola_ctx *ctx, lola_plan *p, const lola_request *reqs, uint32_t n, lola_stream stream) {
    if (!ctx || !p || (!reqs && n)) return set_error(LOLA_E_INVAL, "null argument");
    if (n == 0) return LOLA_OK;
    if (ctx->timing) return set_error(LOLA_E_INVAL, "kernel timing and graph replay are exclusive");
    hipStream_t s = (hipStream_t)stream;
    if (!s) return set_error(LOLA_E_INVAL, "graph replay needs a non-default stream");
    // the same lanes as lola_evaluate (kernel timing is off here)
    const uint32_t n_lanes = (n >= EXEC_LANE_MIN_REQUESTS && p->max_lanes >= 2) ? 2 : 1;
    int rc = prepare(ctx, p, reqs, n, s, n_lanes);
    if (rc) return rc;
    if (!p->graph_valid) {
        if (n_lanes == 2 && (rc = ensure_side(p))) return rc;
        LOLA_HIP(hipStreamSynchronize(s));   // blob upload done before capture
        LOLA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        rc = run_lanes(ctx, p, n_lanes, s);
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
