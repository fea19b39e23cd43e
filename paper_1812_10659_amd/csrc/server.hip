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
//
// A model may also hold a solo plan (the same network compiled for one
// request alone: more rotations in fewer levels) with one slot of its own.  A
// request that arrives to an idle model, with keys for the solo plan, runs
// under it; requests arriving meanwhile run under the model's plan, and their
// waves share the rounds with the solo request's.
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
    std::vector<const uint32_t *> gk, gk_solo, in;   // gk_solo: keys of the solo plan, or empty
    std::vector<uint32_t *> out;
    lola_request view(bool solo) const {
        return lola_request{rlk, solo ? gk_solo.data() : gk.data(), in.data(), out.data()};
    }
};

struct Slot {
    const lola_plan *plan = nullptr;   // the model's plan, or its solo plan for the solo slot
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
    lola_plan *solo = nullptr;      // plan for a request alone (optional), run in solo_slot
    Slot solo_slot;
    uint32_t *ws_solo = nullptr;
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
    std::vector<std::pair<uint64_t, uint32_t>> completed;   // (tag, plan form) since the last poll
    uint64_t rounds = 0;
};

namespace lola {
namespace {

int retire(Model &m, std::vector<std::pair<uint64_t, uint32_t>> &completed, bool wait_one) {
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
    auto done = [&](Slot &s, uint32_t form) {
        if (s.busy && s.finished && s.finish_round <= m.done_round) {
            completed.emplace_back(s.req.tag, form);
            s.busy = false;
            s.finished = false;
        }
    };
    for (Slot &s : m.slots) done(s, LOLA_SERVED_PLAN);
    if (m.solo) done(m.solo_slot, LOLA_SERVED_SOLO);
    return LOLA_OK;
}

int round_model(lola_server *srv, Model &m) {
    // a lone request to an idle model runs under the solo plan, in its slot
    if (m.solo && !m.solo_slot.busy && m.queue.size() == 1 && !m.queue.front().gk_solo.empty()) {
        bool idle = true;
        for (const Slot &s : m.slots) idle = idle && !(s.busy && !s.finished);
        if (idle) {
            Slot &s = m.solo_slot;
            s.busy = true;
            s.finished = false;
            s.level = 1;
            s.req = std::move(m.queue.front());
            m.queue.pop_front();
            s.rq = s.req.view(true);
        }
    }
    // admission into free slots (each slot's footprint was reserved at registration)
    for (Slot &s : m.slots) {
        if (m.queue.empty()) break;
        if (s.busy) continue;
        s.busy = true;
        s.finished = false;
        s.level = 1;
        s.req = std::move(m.queue.front());
        m.queue.pop_front();
        s.rq = s.req.view(false);
    }
    std::vector<Slot *> active, finishing;
    if (m.solo && m.solo_slot.busy && !m.solo_slot.finished) active.push_back(&m.solo_slot);
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
        const lola_plan *p = s.plan;
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
            int rc = emit_level(m.ctx, s.plan, rv, s.level, jobs[n_lanes == 2 && k >= half ? 1 : 0]);
            if (rc) return rc;
            if (++s.level > s.plan->n_waves) finishing.push_back(&s);
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
        if (m.ws_solo) (void)hipFree(m.ws_solo);
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
        m.slots[k].plan = plan;
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

int lola_server_set_solo_plan(lola_server *srv, uint32_t model_id, lola_plan *solo) {
    if (!srv || !solo || model_id >= srv->models.size()) return set_error(LOLA_E_INVAL, "bad argument");
    Model &m = srv->models[model_id];
    if (m.solo) return set_error(LOLA_E_INVAL, "the model already has a solo plan");
    if (solo->loaded_for != m.ctx) return set_error(LOLA_E_INVAL, "solo plan not loaded on the model's context");
    if (!m.queue.empty()) return set_error(LOLA_E_INVAL, "requests already submitted");
    for (const Slot &s : m.slots)
        if (s.busy) return set_error(LOLA_E_INVAL, "requests already submitted");
    // the same request buffers and result layout as the model's plan
    const lola_plan *p = m.plan;
    if (solo->n_inputs != p->n_inputs || solo->outputs.size() != p->outputs.size() ||
        solo->input_map != p->input_map || solo->output_map != p->output_map)
        return set_error(LOLA_E_SHAPE, "solo plan takes other inputs or gives other outputs");
    const size_t N = m.ctx->N, L = m.ctx->L, CT = 2 * L * N, CT3 = 3 * L * N;
    const uint32_t nsq = std::max<uint32_t>(solo->max_squares_per_wave, 1);
    const size_t words = solo->n_phys * CT + nsq * CT3 + (size_t)solo->max_hoist_per_wave * ks_hoist_words(m.ctx);
    if (srv->budget < srv->used + words * 4) return set_error(LOLA_E_NOMEM, "HBM budget too small for the solo slot");
    if (hipMalloc(&m.ws_solo, words * 4) != hipSuccess) return set_error(LOLA_E_NOMEM, "solo slot allocation failed");
    Slot &s = m.solo_slot;
    s.plan = solo;
    s.regs = m.ws_solo;
    s.sq = s.regs + solo->n_phys * CT;
    s.hoist = s.sq + nsq * CT3;
    m.solo = solo;
    srv->used += words * 4;
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

int lola_server_submit_ex(lola_server *srv, uint32_t model_id, const lola_request *req,
                          const uint32_t *const *solo_gk_dev, uint64_t tag) {
    if (!srv || !req || model_id >= srv->models.size()) return set_error(LOLA_E_INVAL, "bad argument");
    Model &m = srv->models[model_id];
    int rc = validate_request(m.plan, *req);
    if (rc) return rc;
    Pending pd;
    if (solo_gk_dev && m.solo) {
        lola_request rs = *req;
        rs.gk_dev = solo_gk_dev;
        if ((rc = validate_request(m.solo, rs))) return rc;
        pd.gk_solo.assign(solo_gk_dev, solo_gk_dev + m.solo->galois.size());
        if (pd.gk_solo.empty()) pd.gk_solo.push_back(nullptr);   // a solo plan without rotations still marks the request
    }
    pd.tag = tag;
    pd.rlk = req->rlk_dev;
    pd.gk.assign(req->gk_dev, req->gk_dev + m.plan->galois.size());
    pd.in.assign(req->in_dev, req->in_dev + m.plan->n_inputs);
    pd.out.assign(req->out_dev, req->out_dev + m.plan->outputs.size());
    m.queue.push_back(std::move(pd));
    return LOLA_OK;
}

int lola_server_submit(lola_server *srv, uint32_t model_id, const lola_request *req, uint64_t tag) {
    return lola_server_submit_ex(srv, model_id, req, nullptr, tag);
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
        if (m.solo) n += m.solo_slot.busy ? 1u : 0u;
    }
    if (pending) *pending = n;
    return LOLA_OK;
}

int lola_server_poll_ex(lola_server *srv, uint64_t *tags, uint32_t *forms, uint32_t cap, uint32_t *n) {
    if (!srv || !n || (!tags && cap)) return set_error(LOLA_E_INVAL, "null argument");
    for (Model &m : srv->models) {
        int rc = retire(m, srv->completed, false);
        if (rc) return rc;
    }
    const uint32_t k = (uint32_t)std::min<size_t>(cap, srv->completed.size());
    for (uint32_t i = 0; i < k; ++i) {
        tags[i] = srv->completed[i].first;
        if (forms) forms[i] = srv->completed[i].second;
    }
    srv->completed.erase(srv->completed.begin(), srv->completed.begin() + k);
    *n = k;
    return LOLA_OK;
}

int lola_server_poll(lola_server *srv, uint64_t *tags, uint32_t cap, uint32_t *n) {
    return lola_server_poll_ex(srv, tags, nullptr, cap, n);
}

}  // extern "C"
