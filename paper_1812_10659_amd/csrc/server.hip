// Serving loop with continuous batching.
//
// A model is a loaded plan on its context (one ring size each).  Each model
// owns a stream, a pool of request slots (register file + square temporaries
// per slot) sized by the HBM budget, and its own scratch.  A scheduling round
// admits queued requests into free slots, then, per model, gathers the next
// wave of every in-flight request -- requests at different depths of the plan
// share the round -- and issues it as one batched launch set on the model's
// stream.  Models of different ring sizes run on separate streams, so their
// work overlaps on the device.  With SRV_LANE_MIN or more requests in flight
// a model's round runs as two lanes: half of its requests on a second stream
// forked from and joined back to the model's stream within the round, so one
// half's kernels fill the other's launch tails.  A request's slot is
// released when the event recorded after its last wave has completed.
#include <chrono>
#include <deque>

#include "plan.hpp"

namespace lola {
namespace {

constexpr uint32_t SRV_KS_CHUNK = 256;
constexpr uint32_t SRV_MUL_CHUNK = 16;
constexpr uint32_t SRV_LOOKAHEAD = 2;   // rounds in flight per model
constexpr uint32_t SRV_LANE_MIN = 16;   // requests in flight from which a round runs as two lanes
constexpr uint32_t SRV_SOLO_WAVES = 8;  // waves a lone request takes per round

struct Pending {
    uint64_t tag;
    const uint32_t *rlk;
    std::vector<const uint32_t *> gk, in;
    std::vector<uint32_t *> out;
    lola_request view() const {
        return lola_request{rlk, gk.data(), in.data(), out.data()};
    }
};

struct Slot {
    bool busy = false;
    bool finished = false;      // last wave issued; waiting for its round event
    uint64_t finish_round = 0;
    uint32_t level = 0;
    Pending req;
    lola_request rq{};
    uint32_t *regs = nullptr, *sq = nullptr, *hoist = nullptr;
};

struct Model {
    lola_ctx *ctx = nullptr;
    lola_plan *plan = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t stream2 = nullptr;  // second lane (models granted SRV_LANE_MIN or more slots)
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    uint32_t *ws = nullptr;         // slots' registers and temporaries, then scratch (two with two lanes)
    uint32_t *scratch = nullptr, *scratch2 = nullptr;
    size_t footprint_bytes = 0;     // per slot
    std::vector<Slot> slots;
    std::deque<Pending> queue;
    uint64_t round = 0;             // rounds issued
    std::deque<std::pair<uint64_t, hipEvent_t>> inflight;   // (round, event)
    uint64_t done_round = 0;        // every round <= done_round has completed
    std::vector<hipEvent_t> free_events;
    uint64_t launched_jobs = 0;
};

}  // namespace
}  // namespace lola

struct lola_server {
    size_t budget = 0, used = 0;
    std::vector<lola::Model> models;
    std::vector<uint64_t> completed;   // tags since the last poll
    uint64_t rounds = 0;
};

namespace lola {
namespace {

int retire(Model &m, std::vector<uint64_t> &completed, bool wait_one) {
    while (!m.inflight.empty()) {
        auto &f = m.inflight.front();
        hipError_t e = wait_one ? hipEventSynchronize(f.second) : hipEventQuery(f.second);
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) return check_hip(e, "server round event");
        m.done_round = f.first;
        m.free_events.push_back(f.second);
        m.inflight.pop_front();
        wait_one = false;
    }
    for (Slot &s : m.slots)
        if (s.busy && s.finished && s.finish_round <= m.done_round) {
            completed.push_back(s.req.tag);
            s.busy = false;
            s.finished = false;
        }
    return LOLA_OK;
}

int round_model(lola_server *srv, Model &m) {
    lola_plan *p = m.plan;
    // admission into free slots (each slot's footprint was reserved at registration)
    for (Slot &s : m.slots) {
        if (m.queue.empty()) break;
        if (s.busy) continue;
        s.busy = true;
        s.finished = false;
        s.level = 1;
        s.req = std::move(m.queue.front());
        m.queue.pop_front();
        s.rq = s.req.view();
    }
    std::vector<Slot *> active, finishing;
    for (Slot &s : m.slots)
        if (s.busy && !s.finished) active.push_back(&s);
    // A lone request (one in flight, none queued) takes up to SRV_SOLO_WAVES
    // waves per round (as many as fit one descriptor slab): with nothing to
    // batch it with, host work between single waves would add to its
    // latency, while a request arriving meanwhile waits at most one such
    // round (about half a millisecond for the MNIST-shaped plan) before the
    // two are batched at their own depths.
    const bool solo = active.size() == 1 && m.queue.empty();
    const uint32_t n_lanes = (!solo && m.stream2 && active.size() >= SRV_LANE_MIN) ? 2 : 1;
    const size_t half = (active.size() + 1) / 2;
    LevelJobs jobs[2];
    Program prog[2];
    size_t n_jobs = 0;
    if (solo) {
        Slot &s = *active[0];
        ReqView rv{&s.rq, s.regs, s.sq, s.hoist};
        for (uint32_t w = 0; w < SRV_SOLO_WAVES && s.level <= p->n_waves; ++w) {
            LevelJobs lj;
            int rc = emit_level(m.ctx, p, rv, s.level, lj);
            if (rc) return rc;
            Program one;
            program_level(m.ctx, one, lj, m.scratch, SRV_KS_CHUNK, SRV_MUL_CHUNK);
            if (!prog[0].launches.empty() && prog[0].blob.size() + one.blob.size() + 256 > lola_ctx::RING_SLAB) break;
            append_program(prog[0], one);
            n_jobs += lj.count();
            ++s.level;
        }
        if (s.level > p->n_waves) finishing.push_back(&s);
    } else {
        for (size_t k = 0; k < active.size(); ++k) {
            Slot &s = *active[k];
            ReqView rv{&s.rq, s.regs, s.sq, s.hoist};
            int rc = emit_level(m.ctx, p, rv, s.level, jobs[n_lanes == 2 && k >= half ? 1 : 0]);
            if (rc) return rc;
            if (++s.level > p->n_waves) finishing.push_back(&s);
        }
        n_jobs = jobs[0].count() + jobs[1].count();
    }
    if (n_jobs == 0) return LOLA_OK;
    while (m.inflight.size() >= SRV_LOOKAHEAD) {
        int rc = retire(m, srv->completed, true);
        if (rc) return rc;
    }
    void *blob[2] = {nullptr, nullptr};
    for (uint32_t l = 0; l < n_lanes; ++l) {
        if (!solo)
            program_level(m.ctx, prog[l], jobs[l], l ? m.scratch2 : m.scratch, SRV_KS_CHUNK, SRV_MUL_CHUNK);
        // both lanes' descriptors go up on the model's stream before the fork,
        // so the descriptor ring's reuse events (recorded on that stream, after
        // this round's join) cover the second lane's reads too
        if (!prog[l].launches.empty()) {
            int rc = desc_upload(m.ctx, prog[l].blob.data(), prog[l].blob.size(), m.stream, &blob[l]);
            if (rc) return rc;
        }
    }
    int rc = LOLA_OK;
    if (n_lanes == 1) {
        rc = program_run(m.ctx, prog[0], (const uint8_t *)blob[0], m.stream);
    } else {
        LOLA_HIP(hipEventRecord(m.fork_ev, m.stream));
        LOLA_HIP(hipStreamWaitEvent(m.stream2, m.fork_ev, 0));
        rc = run_two(m.ctx, prog[0], (const uint8_t *)blob[0], m.stream, prog[1], (const uint8_t *)blob[1],
                     m.stream2);
        // join even after an error, so the model's stream never runs ahead
        LOLA_HIP(hipEventRecord(m.join_ev, m.stream2));
        LOLA_HIP(hipStreamWaitEvent(m.stream, m.join_ev, 0));
    }
    if (rc) return rc;
    m.launched_jobs += n_jobs;
    hipEvent_t ev;
    if (m.free_events.empty()) LOLA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    else { ev = m.free_events.back(); m.free_events.pop_back(); }
    LOLA_HIP(hipEventRecord(ev, m.stream));
    ++m.round;
    m.inflight.emplace_back(m.round, ev);
    for (Slot *s : finishing) {
        s->finished = true;
        s->finish_round = m.round;
    }
    return LOLA_OK;
}

}  // namespace
}  // namespace lola

using namespace lola;

extern "C" {

int lola_server_create(size_t hbm_budget_bytes, lola_server **out) {
    if (!out) return set_error(LOLA_E_INVAL, "null argument");
    *out = new lola_server();
    (*out)->budget = hbm_budget_bytes;
    return LOLA_OK;
}

void lola_server_destroy(lola_server *srv) {
    if (!srv) return;
    for (Model &m : srv->models) {
        if (m.stream) (void)hipStreamSynchronize(m.stream);   // joined with stream2 every round
        if (m.stream2) (void)hipStreamSynchronize(m.stream2);
        for (auto &f : m.inflight) (void)hipEventDestroy(f.second);
        for (hipEvent_t e : m.free_events) (void)hipEventDestroy(e);
        if (m.fork_ev) (void)hipEventDestroy(m.fork_ev);
        if (m.join_ev) (void)hipEventDestroy(m.join_ev);
        if (m.ws) (void)hipFree(m.ws);
        if (m.stream) (void)hipStreamDestroy(m.stream);
        if (m.stream2) (void)hipStreamDestroy(m.stream2);
    }
    delete srv;
}

int lola_server_add_model(lola_server *srv, lola_ctx *ctx, lola_plan *plan, uint32_t max_inflight, uint32_t *model_id) {
    if (!srv || !ctx || !plan || !model_id || max_inflight == 0) return set_error(LOLA_E_INVAL, "null argument");
    if (plan->loaded_for != ctx) return set_error(LOLA_E_INVAL, "plan not loaded on this context");
    const size_t N = ctx->N, L = ctx->L, CT = 2 * L * N, CT3 = 3 * L * N;
    const uint32_t nsq = std::max<uint32_t>(plan->max_squares_per_wave, 1);
    const size_t slot_words = plan->n_phys * CT + nsq * CT3 + (size_t)plan->max_hoist_per_wave * ks_hoist_words(ctx);
    const size_t scratch_words = level_scratch_words(ctx, SRV_KS_CHUNK, SRV_MUL_CHUNK);
    const size_t avail = srv->budget > srv->used ? srv->budget - srv->used : 0;
    if (avail < (scratch_words + slot_words) * 4)
        return set_error(LOLA_E_NOMEM, "HBM budget too small for one request of this model");
    uint32_t fit = (uint32_t)std::min<size_t>(max_inflight, (avail / 4 - scratch_words) / slot_words);
    // a second lane needs a second scratch; it is taken only where the model
    // still gets SRV_LANE_MIN slots beside it
    bool two = false;
    if (fit >= SRV_LANE_MIN && avail / 4 >= 2 * scratch_words + (size_t)SRV_LANE_MIN * slot_words) {
        const uint32_t fit2 = (uint32_t)std::min<size_t>(max_inflight, (avail / 4 - 2 * scratch_words) / slot_words);
        if (fit2 >= SRV_LANE_MIN) {
            fit = fit2;
            two = true;
        }
    }
    Model m;
    m.ctx = ctx;
    m.plan = plan;
    m.footprint_bytes = slot_words * 4;
    const size_t words = fit * slot_words + (two ? 2 : 1) * scratch_words;
    if (hipMalloc(&m.ws, words * 4) != hipSuccess) return set_error(LOLA_E_NOMEM, "server workspace allocation failed");
    LOLA_HIP(hipStreamCreateWithFlags(&m.stream, hipStreamNonBlocking));
    if (two) {
        LOLA_HIP(hipStreamCreateWithFlags(&m.stream2, hipStreamNonBlocking));
        LOLA_HIP(hipEventCreateWithFlags(&m.fork_ev, hipEventDisableTiming));
        LOLA_HIP(hipEventCreateWithFlags(&m.join_ev, hipEventDisableTiming));
    }
    m.slots.resize(fit);
    for (uint32_t k = 0; k < fit; ++k) {
        m.slots[k].regs = m.ws + k * slot_words;
        m.slots[k].sq = m.slots[k].regs + plan->n_phys * CT;
        m.slots[k].hoist = m.slots[k].sq + nsq * CT3;
    }
    m.scratch = m.ws + fit * slot_words;
    if (two) m.scratch2 = m.scratch + scratch_words;
    srv->used += words * 4;
    srv->models.push_back(std::move(m));
    *model_id = (uint32_t)srv->models.size() - 1;
    return LOLA_OK;
}

int lola_server_model_info(const lola_server *srv, uint32_t model_id, uint32_t *slots, uint64_t *footprint_bytes,
                           uint64_t *scratch_bytes, uint64_t *launched_jobs) {
    if (!srv || model_id >= srv->models.size()) return set_error(LOLA_E_INVAL, "bad model id");
    const Model &m = srv->models[model_id];
    if (slots) *slots = (uint32_t)m.slots.size();
    if (footprint_bytes) *footprint_bytes = m.footprint_bytes;
    if (scratch_bytes)
        *scratch_bytes = level_scratch_words(m.ctx, SRV_KS_CHUNK, SRV_MUL_CHUNK) * 4 * (m.stream2 ? 2 : 1);
    if (launched_jobs) *launched_jobs = m.launched_jobs;
    return LOLA_OK;
}

int lola_server_submit(lola_server *srv, uint32_t model_id, const lola_request *req, uint64_t tag) {
    if (!srv || !req || model_id >= srv->models.size()) return set_error(LOLA_E_INVAL, "bad argument");
    Model &m = srv->models[model_id];
    int rc = validate_request(m.plan, *req);
    if (rc) return rc;
    Pending pd;
    pd.tag = tag;
    pd.rlk = req->rlk_dev;
    pd.gk.assign(req->gk_dev, req->gk_dev + m.plan->galois.size());
    pd.in.assign(req->in_dev, req->in_dev + m.plan->n_inputs);
    pd.out.assign(req->out_dev, req->out_dev + m.plan->outputs.size());
    m.queue.push_back(std::move(pd));
    return LOLA_OK;
}

int lola_server_step(lola_server *srv, uint32_t *pending) {
    if (!srv) return set_error(LOLA_E_INVAL, "null argument");
    for (Model &m : srv->models) {
        int rc = retire(m, srv->completed, false);
        if (rc) return rc;
        if ((rc = round_model(srv, m))) return rc;
    }
    ++srv->rounds;
    uint32_t n = 0;
    for (Model &m : srv->models) {
        n += (uint32_t)m.queue.size();
        for (const Slot &s : m.slots) n += s.busy ? 1u : 0u;
    }
    if (pending) *pending = n;
    return LOLA_OK;
}

int lola_server_poll(lola_server *srv, uint64_t *tags, uint32_t cap, uint32_t *n) {
    if (!srv || !n || (!tags && cap)) return set_error(LOLA_E_INVAL, "null argument");
    for (Model &m : srv->models) {
        int rc = retire(m, srv->completed, false);
        if (rc) return rc;
    }
    const uint32_t k = (uint32_t)std::min<size_t>(cap, srv->completed.size());
    std::copy(srv->completed.begin(), srv->completed.begin() + k, tags);
    srv->completed.erase(srv->completed.begin(), srv->completed.begin() + k);
    *n = k;
    return LOLA_OK;
}

}  // extern "C"
