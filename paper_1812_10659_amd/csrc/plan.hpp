// Plan IR: the op list a layer list is lowered to, with wave levels and
// physical register assignment, plus the executor's bound state.
#pragma once
#include <map>
#include <string>
#include <vector>

#include "program.hpp"

namespace lola {

enum OpKind : int { OP_LINCOMB, OP_MULPLAIN, OP_ADDPLAIN, OP_ROTADD, OP_ROT, OP_SQUARE };

struct Op {
    int kind = OP_LINCOMB;
    int dst = -1;
    int src = -1;                 // MULPLAIN / ADDPLAIN / ROT / ROTADD (rotated) / SQUARE
    int addend = -1;              // ROTADD
    std::vector<int> srcs;        // LINCOMB
    std::vector<int64_t> w;       // LINCOMB scalars
    int cmul = -1, cadd = -1;     // plaintext constants (mul form, add form)
    int32_t step = 0;             // rotation step (LOLA_ROW_SWAP for the row swap)
    uint32_t galois = 0;
    bool hoist = false;           // ROT: shares its source's decomposition with the other hoisted
                                  // rotations of that source in its wave
    int level = 0;
};

}  // namespace lola

namespace lola {
// Device state of one execution lane: the program bound for a set of
// requests, its workspace (registers, square temporaries, scratch) and its
// launch descriptors.
struct ExecLane {
    uint32_t *d_ws = nullptr;
    size_t ws_words = 0;
    uint8_t *d_blob = nullptr, *h_blob = nullptr;
    size_t blob_cap = 0;
    std::vector<std::vector<const uint32_t *>> bound_ptrs;   // request pointer sets of the last bind
    Program prog;
    bool prog_valid = false;
};
}  // namespace lola

struct lola_plan {
    uint32_t N = 0, L = 0, t = 0;
    uint32_t K = 1;   // special primes of key switching (digits of K ciphertext primes)
    uint32_t n_inputs = 0, queries = 1;
    uint32_t recipe = 3;                        // LOLA_RECIPE_*
    uint32_t sums = 1;                          // LOLA_SUMS_SEQUENTIAL or LOLA_SUMS_HOISTED
    float predicted_us = 0;                     // cost model, one request inside a large batch
    float predicted_latency_us = 0;             // cost model, one request alone
    uint32_t n_regs = 0;                        // virtual registers (SSA)
    std::vector<lola::Op> ops;                  // in emission order
    std::vector<int> outputs;                   // output registers
    std::vector<std::vector<int64_t>> consts;   // dense slot vectors, N each
    std::vector<uint8_t> const_mul, const_add;  // usage of each constant
    std::map<std::vector<int64_t>, int> const_index;
    std::vector<uint32_t> galois;               // distinct Galois elements, sorted
    std::vector<int32_t> input_map, output_map;
    // scheduling
    uint32_t n_waves = 0;
    std::vector<int> phys;                      // virtual -> physical register (-1: input/output)
    uint32_t n_phys = 0;
    uint32_t max_squares_per_wave = 0;
    uint32_t max_hoist_per_wave = 0;            // distinct sources of hoisted rotations in one wave
    std::vector<std::vector<int>> level_ops;    // op indices of each wave (index = level)
    // loaded constants (device)
    const lola_ctx *loaded_for = nullptr;
    std::vector<uint32_t *> d_cmul, d_cadd;
    std::vector<uint32_t *> d_wtab;             // per op: lincomb scalar table [n_src][2][L]
    // bound evaluation state: a batch runs as one lane on the caller's stream
    // or as two lanes (halves of the batch), the second on side_stream, forked
    // from and joined back to the caller's stream with events
    lola::ExecLane lanes[2];
    uint32_t max_lanes = 2;                     // lola_plan_set_lanes
    hipStream_t side_stream = nullptr;          // non-blocking, default priority
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    hipGraph_t graph = nullptr;                 // captured from lane 0 (one lane)
    hipGraphExec_t graph_exec = nullptr;
    bool graph_valid = false;
};

namespace lola {

// One request's buffers inside an executor: caller-owned inputs / outputs and
// keys (the request) plus its register file and square temporaries.
struct ReqView {
    const lola_request *req;
    uint32_t *regs;      // n_phys ciphertexts
    uint32_t *sq;        // max_squares_per_wave size-3 ciphertexts
    uint32_t *hoist;     // max_hoist_per_wave hoist areas (ks_hoist_words each)
};

// The jobs of one wave, gathered over any number of requests.
struct LevelJobs {
    std::vector<LinJob> lin;
    std::vector<PlainJob> plain;
    std::vector<KsJob> ks, relin;
    std::vector<KsJob> hsrc, hrot;   // hoisted rotations: sources, then the rotations
    std::vector<MulJob> muls;
    size_t count() const { return lin.size() + plain.size() + ks.size() + muls.size() + hrot.size(); }
};

// Appends the jobs of plan level `level` for one request.
int emit_level(const lola_ctx *ctx, const lola_plan *p, const ReqView &rv, uint32_t level, LevelJobs &out);
// Appends the launches of gathered jobs to a program (key switches and
// products chunked over the given scratch).
void program_level(const lola_ctx *ctx, Program &prog, LevelJobs &jobs, uint32_t *scratch, uint32_t ks_chunk,
                   uint32_t mul_chunk);
// Scratch words that program_level needs for chunk sizes ks_chunk / mul_chunk.
size_t level_scratch_words(const lola_ctx *ctx, uint32_t ks_chunk, uint32_t mul_chunk);
// Two programs (descriptors already on the device at da / db) on two
// streams, interleaved launch by launch.
int run_two(lola_ctx *ctx, const Program &a, const uint8_t *da, hipStream_t sa, const Program &b,
            const uint8_t *db, hipStream_t sb);
// Checks a request's arrays against the plan (keys, inputs, outputs, aliasing).
int validate_request(const lola_plan *p, const lola_request &r);

}  // namespace lola
