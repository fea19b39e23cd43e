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
    int level = 0;
};

}  // namespace lola

struct lola_plan {
    uint32_t N = 0, L = 0, t = 0;
    uint32_t n_inputs = 0, queries = 1;
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
    // loaded constants (device)
    const lola_ctx *loaded_for = nullptr;
    std::vector<uint32_t *> d_cmul, d_cadd;
    // bound evaluation state
    uint32_t *d_ws = nullptr;                   // registers + square temporaries + scratch
    size_t ws_words = 0;
    uint8_t *d_blob = nullptr, *h_blob = nullptr;
    size_t blob_cap = 0;
    std::vector<std::vector<const uint32_t *>> bound_ptrs;   // request pointer sets of the last bind
    lola::Program prog;
    bool prog_valid = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_valid = false;
    // device arrays referenced by LinJob (pointer lists and scalar tables)
    std::vector<uint64_t> lin_aux;              // packed into the blob at bind time
};
