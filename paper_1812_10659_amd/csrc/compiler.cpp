// Layer compiler: lowers a layer list to an op list with the paper's vector
// representations and matrix-vector recipes (Sec. 4.2), then levels the ops
// into waves of independent work and assigns physical registers.
//
// Recipes (W: weights, values modulo t):
//   convolution vector - row major (Sec. 4.2.2): the input is k*k messages,
//     message a*k+b holding input[stride*y + a][stride*x + b] at slot y*n+x;
//     map m is sum_{a,b} w[m][a][b] * message(a,b) (+ bias), one message per
//     map, values at slots 0..n*n-1 (dense);
//   combining messages (Table 1, "combine ... using rotations"): message j is
//     rotated right by j*unit and added; built as a binary tree so only
//     log2(count) distinct rotation keys are needed;
//   stacked vector - row major (Sec. 4.2.2): copies of a dense vector at
//     stride P (next power of two >= its length) are made by rotate-and-add
//     over -P, -2P, ..., -N/4 and the row swap; each round multiplies by rows
//     laid out one per block, sums each block by rotations 1..P/2, keeps the
//     block's first slot (mask) and adds the bias; rounds are then combined
//     into an interleaved vector (value C*rho + c at slot P*c + rho); as the
//     last layer (convolution, square, dense) a single round without mask
//     is the output, value o at slot P*o;
//   interleaved vector - row major (Sec. 4.2.2): per output, a product with
//     the row permuted to the interleaved layout and a rotate-and-sum that
//     collects every occupied slot into slot 0 (sparse output);
//   dense vector - row major (Sec. 4.2.2): per output row, product with the
//     row in every query block, rotate-and-sum over the block, mask, then
//     combination into an interleaved vector (value j of query q at P*q + j);
//     in chains of dense layers, the row's product summed over the whole
//     message (rotations 1 .. N/4 and the row swap) so that every slot holds
//     the output: one message per row (sparse output);
//   sparse vector - column major (Sec. 4.2.2): on a sparse input (message i
//     holds v_i in every slot), W v = sum_i v_i c^i, one product of message i
//     with column i laid out at slots 0..r-1 per input, summed: a dense
//     output with no rotation.  The two-convolution network's gather of its
//     sparse outputs into one message is this recipe with W = I.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>

#include "plan.hpp"

namespace lola {
namespace {

uint32_t next_pow2(uint32_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct Builder {
    lola_plan *p;
    // Hoisted sums (the latency layout, LOLA_SUMS_HOISTED): rotate_and_sum
    // takes its steps in groups of up to three consecutive steps other than
    // the row swap; a group is the 2^k - 1 rotations of the current message by
    // the group's subset sums, all hoisted (one decomposition), added to it in
    // one linear combination: one level instead of k.  combine_tree becomes
    // one level too: every member after the first rotated by its own offset,
    // then one linear combination.  The slots are those of the sequential
    // forms (rotations within a row compose additively).
    bool hoist_sums = false;
    int reg() { return (int)p->n_regs++; }
    int cst(std::vector<int64_t> v, bool mul) {
        for (auto &x : v) {
            x %= (int64_t)p->t;
            if (x < 0) x += p->t;
        }
        auto it = p->const_index.find(v);
        int id;
        if (it == p->const_index.end()) {
            id = (int)p->consts.size();
            p->const_index.emplace(v, id);
            p->consts.push_back(std::move(v));
            p->const_mul.push_back(0);
            p->const_add.push_back(0);
        } else {
            id = it->second;
        }
        (mul ? p->const_mul : p->const_add)[id] = 1;
        return id;
    }
    std::vector<int64_t> zeros() const { return std::vector<int64_t>(p->N, 0); }
    int lincomb(const std::vector<int> &srcs, const std::vector<int64_t> &w, int cadd) {
        Op o;
        o.kind = OP_LINCOMB;
        o.dst = reg();
        o.srcs = srcs;
        o.w = w;
        o.cadd = cadd;
        p->ops.push_back(o);
        return o.dst;
    }
    int mulplain(int src, int cmul, int cadd = -1) {
        Op o;
        o.kind = OP_MULPLAIN;
        o.dst = reg();
        o.src = src;
        o.cmul = cmul;
        o.cadd = cadd;
        p->ops.push_back(o);
        return o.dst;
    }
    int addplain(int src, int cadd) {
        Op o;
        o.kind = OP_ADDPLAIN;
        o.dst = reg();
        o.src = src;
        o.cadd = cadd;
        p->ops.push_back(o);
        return o.dst;
    }
    // addend + rotate(src, step)
    int rotadd(int src, int32_t step, int addend) {
        Op o;
        o.kind = OP_ROTADD;
        o.dst = reg();
        o.src = src;
        o.addend = addend;
        o.step = step;
        o.galois = lola_galois_element(p->N, step);
        p->ops.push_back(o);
        return o.dst;
    }
    // hoist: the rotation shares its source's decomposition with the other
    // hoisted rotations of that source in its wave
    int rot(int src, int32_t step, bool hoist = false) {
        Op o;
        o.kind = OP_ROT;
        o.dst = reg();
        o.src = src;
        o.step = step;
        o.galois = lola_galois_element(p->N, step);
        o.hoist = hoist;
        p->ops.push_back(o);
        return o.dst;
    }
    int square(int src) {
        Op o;
        o.kind = OP_SQUARE;
        o.dst = reg();
        o.src = src;
        p->ops.push_back(o);
        return o.dst;
    }
    int rotate_and_sum(int src, const std::vector<int32_t> &steps) {
        int cur = src;
        if (!hoist_sums) {
            for (int32_t k : steps) cur = rotadd(cur, k, cur);
            return cur;
        }
        size_t i = 0;
        while (i < steps.size()) {
            std::vector<int32_t> grp;
            while (i < steps.size() && steps[i] != LOLA_ROW_SWAP && grp.size() < 3) grp.push_back(steps[i++]);
            if (grp.size() < 2) {   // a row swap or a lone step: a fused rotate-and-add
                cur = rotadd(cur, grp.empty() ? steps[i++] : grp[0], cur);
                continue;
            }
            std::vector<int> terms{cur};
            for (uint32_t m = 1; m < (1u << grp.size()); ++m) {
                int32_t a = 0;
                for (size_t k = 0; k < grp.size(); ++k)
                    if (m >> k & 1) a += grp[k];
                terms.push_back(rot(cur, a, true));
            }
            cur = lincomb(terms, std::vector<int64_t>(terms.size(), 1), -1);
        }
        return cur;
    }
    // sum_k w[k] * srcs[k] (+ cadd) for any number of sources: linear
    // combinations of at most LIN_MAX sources, each later one taking the
    // previous partial sum as its first source (weight 1)
    int lincomb_any(const std::vector<int> &srcs, const std::vector<int64_t> &w, int cadd) {
        size_t k = std::min<size_t>(srcs.size(), LIN_MAX);
        int acc = lincomb(std::vector<int>(srcs.begin(), srcs.begin() + k),
                          std::vector<int64_t>(w.begin(), w.begin() + k), cadd);
        while (k < srcs.size()) {
            const size_t m = std::min<size_t>(srcs.size() - k, LIN_MAX - 1);
            std::vector<int> s2{acc};
            std::vector<int64_t> w2{1};
            s2.insert(s2.end(), srcs.begin() + k, srcs.begin() + k + m);
            w2.insert(w2.end(), w.begin() + k, w.begin() + k + m);
            acc = lincomb(s2, w2, -1);
            k += m;
        }
        return acc;
    }
    // Sparse vector - column major: one term v_i c^i (the sparse message of
    // input i times column i as a plaintext), then the sum of the terms with
    // an optional add-form constant (the bias at the output slots).
    int column_term(int sparse_src, std::vector<int64_t> column) { return mulplain(sparse_src, cst(std::move(column), true)); }
    int column_sum(const std::vector<int> &terms, int cadd) {
        return lincomb_any(terms, std::vector<int64_t>(terms.size(), 1), cadd);
    }
    int combine_tree(std::vector<int> regs, int32_t unit) {
        if (hoist_sums && regs.size() > 2) {
            std::vector<int> terms{regs[0]};
            for (size_t j = 1; j < regs.size(); ++j) terms.push_back(rot(regs[j], -unit * (int32_t)j));
            return lincomb_any(terms, std::vector<int64_t>(terms.size(), 1), -1);
        }
        int32_t stride = unit;
        while (regs.size() > 1) {
            std::vector<int> nxt;
            for (size_t i = 0; i < regs.size(); i += 2) {
                if (i + 1 < regs.size())
                    nxt.push_back(rotadd(regs[i + 1], -stride, regs[i]));
                else
                    nxt.push_back(regs[i]);
            }
            regs.swap(nxt);
            stride *= 2;
        }
        return regs[0];
    }
};

int unsupported(const std::string &m) { return set_error(LOLA_E_UNSUPPORTED, m); }

int64_t bias_at(const lola_layer &l, int j) { return l.bias ? l.bias[j] : 0; }

// ---- network families -------------------------------------------------
// shared: the two dense layers of the five-layer network with one shared
// reduction tail and a packed output message (LOLA_RECIPE_SHARED_REDUCTION);
// otherwise every stacked round is summed over its whole block and each
// output gets its own message (LOLA_RECIPE_FULL_REDUCTION).
// A vector between layers: sparse (value i in every slot of message regs[i])
// or dense (value i at slot pos[i] of the one message regs[0]).
struct ChainVec {
    std::vector<int> regs;
    bool sparse = false;
    std::vector<uint32_t> pos;
    int width = 0;
};

// DENSE and SQUARE layers ls[from..n) on v, each dense layer with the recipe
// its input's representation calls for (Sec. 4.2.2): dense vector - row
// major on a dense input (per row, the product with the row laid out at the
// input's slots, then a rotate-and-sum over every slot: a sparse result) and
// sparse vector - column major on a sparse input (the sum of v_i c^i, no
// rotation: a dense result, value j at slot j); a square acts on every
// message of the representation.
int emit_chain(Builder &b, const lola_layer *ls, uint32_t from, uint32_t n, ChainVec &v) {
    const uint32_t N = b.p->N;
    int dim = v.width;
    for (uint32_t l = from; l < n; ++l) {
        if (ls[l].kind == LOLA_LAYER_SQUARE) continue;
        if (ls[l].kind != LOLA_LAYER_DENSE) return unsupported("a chain holds DENSE and SQUARE layers");
        if (ls[l].in_dim != dim || ls[l].out_dim <= 0 || !ls[l].weight)
            return unsupported("dense layer sizes must chain");
        if ((uint32_t)ls[l].in_dim > N || (uint32_t)ls[l].out_dim > N)
            return unsupported("dense layer larger than a message");
        dim = ls[l].out_dim;
    }
    std::vector<int32_t> full;
    for (uint32_t s = 1; s < N / 2; s *= 2) full.push_back((int32_t)s);
    full.push_back(LOLA_ROW_SWAP);
    for (uint32_t l = from; l < n; ++l) {
        const lola_layer &ly = ls[l];
        if (ly.kind == LOLA_LAYER_SQUARE) {
            for (int &x : v.regs) x = b.square(x);
            continue;
        }
        const int in = ly.in_dim, r = ly.out_dim;
        if (v.sparse) {
            std::vector<int> terms;
            for (int i = 0; i < in; ++i) {
                auto col = b.zeros();
                for (int j = 0; j < r; ++j) col[j] = ly.weight[(size_t)j * in + i];
                terms.push_back(b.column_term(v.regs[i], std::move(col)));
            }
            int cadd = -1;
            if (ly.bias) {
                auto bv = b.zeros();
                for (int j = 0; j < r; ++j) bv[j] = ly.bias[j];
                cadd = b.cst(bv, false);
            }
            v.regs = {b.column_sum(terms, cadd)};
            v.pos.resize(r);
            for (int j = 0; j < r; ++j) v.pos[j] = (uint32_t)j;
        } else {
            std::vector<int> outs;
            for (int j = 0; j < r; ++j) {
                auto row = b.zeros();
                for (int i = 0; i < in; ++i) row[v.pos[i]] = ly.weight[(size_t)j * in + i];
                int z = b.rotate_and_sum(b.mulplain(v.regs[0], b.cst(row, true)), full);
                if (ly.bias) z = b.addplain(z, b.cst(std::vector<int64_t>(N, ly.bias[j]), false));
                outs.push_back(z);
            }
            v.regs = outs;
            v.pos.clear();
        }
        v.sparse = !v.sparse;
        v.width = r;
    }
    return LOLA_OK;
}

// The plan's outputs: the chain's messages and where each value lies.
void chain_outputs(lola_plan *p, const ChainVec &v) {
    const uint32_t N = p->N;
    p->outputs = v.regs;
    p->output_map.assign((size_t)v.regs.size() * N, -1);
    for (int j = 0; j < v.width; ++j) {
        if (v.sparse) p->output_map[(size_t)j * N] = j;
        else p->output_map[v.pos[j]] = j;
    }
}

int compile_conv_net(lola_plan *p, Builder &b, const lola_layer *ls, uint32_t n, bool shared) {
    // CONV2D (or CONV2D_DENSE_INPUT), SQUARE, DENSE, then any chain of DENSE
    // and SQUARE layers.  SQUARE, DENSE after the first dense layer ends in
    // an interleaved vector - row major output layer (Table 1); other chains
    // continue from the interleaved hidden vector with emit_chain.
    const bool small = n == 3;
    const bool two = n == 5 && ls[3].kind == LOLA_LAYER_SQUARE && ls[4].kind == LOLA_LAYER_DENSE;
    const bool dense_in = ls[0].kind == LOLA_LAYER_CONV2D_DENSE_INPUT;
    if (n < 3 || ls[1].kind != LOLA_LAYER_SQUARE || ls[2].kind != LOLA_LAYER_DENSE)
        return unsupported("convolution networks must be CONV2D, SQUARE, DENSE, then DENSE and SQUARE layers");
    for (uint32_t l = 3; l < n; ++l)
        if (ls[l].kind != LOLA_LAYER_DENSE && ls[l].kind != LOLA_LAYER_SQUARE)
            return unsupported("convolution networks must be CONV2D, SQUARE, DENSE, then DENSE and SQUARE layers");
    const lola_layer &cv = ls[0], &d1 = ls[2], &d2 = ls[two ? 4 : 2];
    const uint32_t N = p->N;
    if (cv.in_h != cv.in_w || cv.k <= 0 || cv.stride <= 0 || cv.maps <= 0 || cv.in_h < cv.k || !cv.weight)
        return unsupported("bad convolution shape");
    const int n_out = (cv.in_h - cv.k) / cv.stride + 1, V = n_out * n_out, K2 = cv.k * cv.k;
    if (K2 > (int)LIN_MAX) return unsupported("convolution window larger than 32 positions");
    if ((uint32_t)(cv.maps * V) > N / 2) return unsupported("convolution output exceeds one slot row");
    const int D = cv.maps * V;
    if (d1.in_dim != D || !d1.weight || d1.out_dim <= 0) return unsupported("first dense layer must take maps*n*n inputs");
    // slot of the first dense layer's input i = m*V + y*n_out + x after the
    // convolution and the combination of the maps
    std::vector<uint32_t> pos((size_t)D);
    uint32_t span = (uint32_t)D;
    std::vector<uint32_t> offs;
    if (dense_in) {
        // window corners at stride*(y*W + x); maps go to the four parity
        // classes of that lattice (stride 2), further ones to bands below
        if (cv.stride != 2 || small) return unsupported("dense-input convolution: stride 2 and layers after the first dense one");
        const uint32_t W = (uint32_t)cv.in_w, band = W * (uint32_t)(2 * n_out);
        const uint32_t cls[4] = {0, 1, W, W + 1};
        for (int m = 0; m < cv.maps; ++m) offs.push_back(cls[m % 4] + band * (uint32_t)(m / 4));
        span = 0;
        for (int m = 0; m < cv.maps; ++m)
            for (int yy = 0; yy < n_out; ++yy)
                for (int xx = 0; xx < n_out; ++xx) {
                    const uint32_t sl = offs[m] + 2 * (uint32_t)yy * W + 2 * (uint32_t)xx;
                    pos[(size_t)m * V + yy * n_out + xx] = sl;
                    span = std::max(span, sl + 1);
                }
        if (span > N / 2) return unsupported("dense-input convolution output exceeds one slot row");
    } else {
        for (int i = 0; i < D; ++i) pos[i] = (uint32_t)i;
    }
    const uint32_t P = next_pow2(span);
    if (P > N / 2) return unsupported("dense input too long to stack");
    const uint32_t C = N / P;
    const uint32_t R = ((uint32_t)d1.out_dim + C - 1) / C;
    if (small && R != 1) return unsupported("a final dense layer after the convolution needs out_dim <= N / next_pow2(in_dim)");
    if (R > P) return unsupported("too many stacked rounds for the interleaved layout");
    if (two && (d2.in_dim != d1.out_dim || !d2.weight || d2.out_dim <= 0))
        return unsupported("second dense layer shape");
    std::vector<int> ins(K2);
    std::vector<uint32_t> corner((size_t)V);   // slot of window (y, x) in the conv messages
    if (dense_in) {
        // input: one dense message, padded pixel (i, j) at slot i*W + j
        // (App. C); message (a, b) of the convolution representation is the
        // input rotated left by a*W + b, times the 0/1 mask of the corners
        const uint32_t W = (uint32_t)cv.in_w;
        if ((uint32_t)(cv.in_h * cv.in_w) > N / 2) return unsupported("dense input longer than a slot row");
        p->n_inputs = 1;
        p->queries = 1;
        p->n_regs = 1;
        p->input_map.assign(N, -1);
        for (int i = 0; i < cv.in_h; ++i)
            for (int j = 0; j < cv.in_w; ++j) p->input_map[(size_t)i * W + j] = i * cv.in_w + j;
        auto mask = b.zeros();
        for (int yy = 0; yy < n_out; ++yy)
            for (int xx = 0; xx < n_out; ++xx) {
                corner[yy * n_out + xx] = 2 * (uint32_t)yy * W + 2 * (uint32_t)xx;
                mask[corner[yy * n_out + xx]] = 1;
            }
        const int cm = b.cst(mask, true);
        for (int a = 0; a < cv.k; ++a)
            for (int c = 0; c < cv.k; ++c) {
                const int32_t r = a * (int32_t)W + c;
                ins[a * cv.k + c] = b.mulplain(r ? b.rot(0, r, true) : 0, cm);
            }
    } else {
        // inputs: convolution representation
        p->n_inputs = (uint32_t)K2;
        p->queries = 1;
        p->n_regs = p->n_inputs;
        p->input_map.assign((size_t)K2 * N, -1);
        for (int a = 0; a < cv.k; ++a)
            for (int c = 0; c < cv.k; ++c)
                for (int y = 0; y < n_out; ++y)
                    for (int x = 0; x < n_out; ++x)
                        p->input_map[(size_t)(a * cv.k + c) * N + y * n_out + x] =
                            (cv.stride * y + a) * cv.in_w + (cv.stride * x + c);
        for (int i = 0; i < K2; ++i) ins[i] = i;
        for (int v = 0; v < V; ++v) corner[v] = (uint32_t)v;
    }
    // convolution: one linear combination per map (+ bias at the window slots)
    std::vector<int> maps;
    for (int m = 0; m < cv.maps; ++m) {
        std::vector<int64_t> w(cv.weight + (size_t)m * K2, cv.weight + (size_t)(m + 1) * K2);
        int cadd = -1;
        if (cv.bias) {
            auto v = b.zeros();
            for (int s = 0; s < V; ++s) v[corner[s]] = cv.bias[m];
            cadd = b.cst(v, false);
        }
        maps.push_back(b.lincomb(ins, w, cadd));
    }
    int y;
    if (dense_in) {
        y = maps[0];
        for (int m = 1; m < cv.maps; ++m) y = b.rotadd(maps[m], -(int32_t)offs[m], y);
    } else {
        y = b.combine_tree(maps, V);
    }
    y = b.square(y);
    // stack C copies at stride P
    std::vector<int32_t> st;
    for (uint32_t s = P; s < N / 2; s *= 2) st.push_back(-(int32_t)s);
    st.push_back(LOLA_ROW_SWAP);
    const int S = b.rotate_and_sum(y, st);
    std::vector<int32_t> blk;
    for (uint32_t s = 1; s < P; s *= 2) blk.push_back((int32_t)s);
    if (small) {
        // one stacked round is the output layer: row o in block o, result o
        // at slot P*o of the single output message
        auto rows = b.zeros(), bias = b.zeros();
        for (int o = 0; o < d1.out_dim; ++o) {
            for (int i = 0; i < D; ++i) rows[P * o + pos[i]] = d1.weight[(size_t)o * D + i];
            bias[P * o] = bias_at(d1, o);
        }
        int z = b.mulplain(S, b.cst(rows, true));
        z = b.rotate_and_sum(z, blk);
        if (d1.bias) z = b.addplain(z, b.cst(bias, false));
        p->outputs.push_back(z);
        p->output_map.assign(N, -1);
        for (int o = 0; o < d1.out_dim; ++o) p->output_map[(size_t)P * o] = o;
        return LOLA_OK;
    }
    // rounds of stacked vector - row major.  Full: each round summed over its
    // block (rotations 1 .. P/2), masked to slot P c with the bias there, and
    // round rho shifted right by rho.  Shared: each round summed only within
    // groups of G = next_pow2(R) slots and masked to the group starts
    // P c + G m (bias at P c); after the shift by rho the rounds fill distinct
    // offsets of those groups, and one rotate-and-sum over G .. P/2 completes
    // every round's block sum at slot P c + rho together.
    const uint32_t G = shared ? next_pow2(R) : P;
    std::vector<int32_t> grp, tail;
    for (uint32_t s = 1; s < G; s *= 2) grp.push_back((int32_t)s);
    for (uint32_t s = G; s < P; s *= 2) tail.push_back((int32_t)s);
    std::vector<int> rounds;
    for (uint32_t rho = 0; rho < R; ++rho) {
        auto rows = b.zeros(), mask = b.zeros(), bias = b.zeros();
        for (uint32_t c = 0; c < C; ++c) {
            const uint32_t j = C * rho + c;
            if (j >= (uint32_t)d1.out_dim) continue;
            for (int i = 0; i < D; ++i) rows[P * c + pos[i]] = d1.weight[(size_t)j * D + i];
            for (uint32_t m = 0; m < P / G; ++m) mask[P * c + G * m] = 1;
            bias[P * c] = bias_at(d1, (int)j);
        }
        int z = b.mulplain(S, b.cst(rows, true));
        z = b.rotate_and_sum(z, grp);
        z = b.mulplain(z, b.cst(mask, true), d1.bias ? b.cst(bias, false) : -1);
        rounds.push_back(z);
    }
    int h = b.combine_tree(rounds, 1);
    if (shared) h = b.rotate_and_sum(h, tail);
    if (!two) {
        // any other chain continues from the interleaved hidden vector,
        // value C rho + c at slot P c + rho
        ChainVec v;
        v.regs = {h};
        v.width = d1.out_dim;
        for (int j = 0; j < d1.out_dim; ++j) v.pos.push_back(P * ((uint32_t)j % C) + (uint32_t)j / C);
        const int rc = emit_chain(b, ls, 3, n, v);
        if (rc) return rc;
        chain_outputs(p, v);
        p->recipe = shared ? LOLA_RECIPE_SHARED_REDUCTION : LOLA_RECIPE_FULL_REDUCTION;
        return LOLA_OK;
    }
    h = b.square(h);
    // interleaved row major: value j = C*rho + c at slot P*c + rho
    const uint32_t GR = next_pow2(R);
    std::vector<int32_t> coll;
    for (uint32_t s = 1; s < GR; s *= 2) coll.push_back((int32_t)s);
    for (uint32_t s = P; s < N / 2 && s < P * C; s *= 2) coll.push_back((int32_t)s);
    if (P * C > N / 2) coll.push_back(LOLA_ROW_SWAP);
    auto out_row = [&](int o, uint32_t shift) {
        auto rows = b.zeros();
        for (uint32_t rho = 0; rho < R; ++rho)
            for (uint32_t c = 0; c < C; ++c) {
                const uint32_t j = C * rho + c;
                if (j < (uint32_t)d1.out_dim) rows[P * c + shift + rho] = d2.weight[(size_t)o * d2.in_dim + j];
            }
        return b.cst(rows, true);
    };
    if (shared) {
        // one packed message: copy o of the input is rotated right by GR*o
        // (all copies hoisted rotations of the input), times row o at offset
        // GR*o of every block; the products are added and one rotate-and-sum
        // leaves output o at slot GR*o
        if ((uint64_t)GR * (uint64_t)d2.out_dim > P) return unsupported("packed output does not fit one stacking block");
        std::vector<int> copies{h}, prods;
        for (int o = 1; o < d2.out_dim; ++o) copies.push_back(b.rot(h, -(int32_t)(GR * (uint32_t)o), true));
        for (int o = 0; o < d2.out_dim; ++o) prods.push_back(b.mulplain(copies[o], out_row(o, GR * (uint32_t)o)));
        int z = b.lincomb_any(prods, std::vector<int64_t>(prods.size(), 1), -1);
        z = b.rotate_and_sum(z, coll);
        if (d2.bias) {
            auto bv = b.zeros();
            for (int o = 0; o < d2.out_dim; ++o) bv[GR * (uint32_t)o] = d2.bias[o];
            z = b.addplain(z, b.cst(bv, false));
        }
        p->outputs.push_back(z);
        p->output_map.assign(N, -1);
        for (int o = 0; o < d2.out_dim; ++o) p->output_map[(size_t)GR * o] = o;
        p->recipe = LOLA_RECIPE_SHARED_REDUCTION;
        return LOLA_OK;
    }
    p->output_map.assign((size_t)d2.out_dim * N, -1);
    for (int o = 0; o < d2.out_dim; ++o) {
        int z = b.mulplain(h, out_row(o, 0));
        z = b.rotate_and_sum(z, coll);
        if (d2.bias) {
            auto bv = b.zeros();
            bv[0] = d2.bias[o];
            z = b.addplain(z, b.cst(bv, false));
        }
        p->outputs.push_back(z);
        p->output_map[(size_t)o * N] = o;
    }
    p->recipe = LOLA_RECIPE_FULL_REDUCTION;
    return LOLA_OK;
}

int compile_stacked_dense(lola_plan *p, Builder &b, const lola_layer *ls, uint32_t n) {
    // DENSE [, SQUARE] with in_dim <= N/4
    const lola_layer &d = ls[0];
    const uint32_t N = p->N;
    if (n > 2 || (n == 2 && ls[1].kind != LOLA_LAYER_SQUARE)) return unsupported("stacked dense: DENSE [, SQUARE]");
    const uint32_t P = next_pow2((uint32_t)d.in_dim), C = N / P;
    if ((uint32_t)d.out_dim > C) return unsupported("stacked dense: more rows than blocks");
    p->n_inputs = 1;
    p->queries = 1;
    p->n_regs = 1;
    p->input_map.assign(N, -1);
    for (uint32_t s = 0; s < N; ++s)
        if ((int)(s % P) < d.in_dim) p->input_map[s] = (int32_t)(s % P);
    auto rows = b.zeros();
    for (int j = 0; j < d.out_dim; ++j)
        for (int i = 0; i < d.in_dim; ++i) rows[P * j + i] = d.weight[(size_t)j * d.in_dim + i];
    int z = b.mulplain(0, b.cst(rows, true));
    std::vector<int32_t> blk;
    for (uint32_t s = 1; s < P; s *= 2) blk.push_back((int32_t)s);
    z = b.rotate_and_sum(z, blk);
    if (d.bias) {
        auto bv = b.zeros();
        for (int j = 0; j < d.out_dim; ++j) bv[P * j] = d.bias[j];
        z = b.addplain(z, b.cst(bv, false));
    }
    if (n == 2) z = b.square(z);
    p->outputs.push_back(z);
    p->output_map.assign(N, -1);
    for (int j = 0; j < d.out_dim; ++j) p->output_map[P * j] = j;
    return LOLA_OK;
}

int compile_dense_head(lola_plan *p, Builder &b, const lola_layer *ls, uint32_t n) {
    // DENSE, SQUARE, DENSE with N/4 < in_dim <= N/2
    if (n != 3 || ls[1].kind != LOLA_LAYER_SQUARE || ls[2].kind != LOLA_LAYER_DENSE)
        return unsupported("dense head must be DENSE, SQUARE, DENSE");
    const lola_layer &d1 = ls[0], &d2 = ls[2];
    const uint32_t N = p->N;
    const uint32_t P = next_pow2((uint32_t)d1.in_dim), Qn = N / P;
    const uint32_t H = (uint32_t)d1.out_dim;
    if (H > P || d2.in_dim != d1.out_dim || !d2.weight) return unsupported("dense head shape");
    p->n_inputs = 1;
    p->queries = Qn;
    p->n_regs = 1;
    p->input_map.assign(N, -1);
    for (uint32_t q = 0; q < Qn; ++q)
        for (int i = 0; i < d1.in_dim; ++i) p->input_map[P * q + i] = (int32_t)(q * d1.in_dim + i);
    std::vector<int32_t> blk;
    for (uint32_t s = 1; s < P; s *= 2) blk.push_back((int32_t)s);
    auto mask = b.zeros();
    for (uint32_t q = 0; q < Qn; ++q) mask[P * q] = 1;
    const int cmask = b.cst(mask, true);
    std::vector<int> hidden;
    for (uint32_t j = 0; j < H; ++j) {
        auto rows = b.zeros();
        for (uint32_t q = 0; q < Qn; ++q)
            for (int i = 0; i < d1.in_dim; ++i) rows[P * q + i] = d1.weight[(size_t)j * d1.in_dim + i];
        int z = b.mulplain(0, b.cst(rows, true));
        z = b.rotate_and_sum(z, blk);
        z = b.mulplain(z, cmask);
        hidden.push_back(z);
    }
    int acc = b.combine_tree(hidden, 1);
    if (d1.bias) {
        auto bv = b.zeros();
        for (uint32_t q = 0; q < Qn; ++q)
            for (uint32_t j = 0; j < H; ++j) bv[P * q + j] = d1.bias[j];
        acc = b.addplain(acc, b.cst(bv, false));
    }
    const int h = b.square(acc);
    std::vector<int32_t> coll;
    for (uint32_t s = 1; s < next_pow2(std::max<uint32_t>(H, 2)); s *= 2) coll.push_back((int32_t)s);
    p->output_map.assign((size_t)d2.out_dim * N, -1);
    for (int o = 0; o < d2.out_dim; ++o) {
        auto rows = b.zeros();
        for (uint32_t q = 0; q < Qn; ++q)
            for (uint32_t j = 0; j < H; ++j) rows[P * q + j] = d2.weight[(size_t)o * d2.in_dim + j];
        int z = b.mulplain(h, b.cst(rows, true));
        z = b.rotate_and_sum(z, coll);
        if (d2.bias) {
            auto bv = b.zeros();
            for (uint32_t q = 0; q < Qn; ++q) bv[P * q] = d2.bias[o];
            z = b.addplain(z, b.cst(bv, false));
        }
        p->outputs.push_back(z);
        for (uint32_t q = 0; q < Qn; ++q) p->output_map[(size_t)o * N + P * q] = (int32_t)(q * d2.out_dim + o);
    }
    return LOLA_OK;
}

int compile_dense_head_stacked(lola_plan *p, Builder &b, const lola_layer *ls, uint32_t n) {
    // DENSE, SQUARE, DENSE with in_dim <= N/2, one query per message: the
    // client sends N/P copies of the input (stacked representation); the
    // hidden layer is stacked vector - row major in rounds, the output layer
    // interleaved vector - row major (value at slot 0)
    if (n != 3 || ls[1].kind != LOLA_LAYER_SQUARE || ls[2].kind != LOLA_LAYER_DENSE)
        return unsupported("dense head must be DENSE, SQUARE, DENSE");
    const lola_layer &d1 = ls[0], &d2 = ls[2];
    const uint32_t N = p->N;
    const uint32_t P = next_pow2((uint32_t)d1.in_dim), C = N / P;
    const uint32_t H = (uint32_t)d1.out_dim, R = (H + C - 1) / C;
    if (C < 2 || R > P || d2.in_dim != d1.out_dim || !d2.weight) return unsupported("stacked head shape");
    p->n_inputs = 1;
    p->queries = 1;
    p->n_regs = 1;
    p->input_map.assign(N, -1);
    for (uint32_t c = 0; c < C; ++c)
        for (int i = 0; i < d1.in_dim; ++i) p->input_map[P * c + i] = i;
    std::vector<int32_t> blk;
    for (uint32_t s = 1; s < P; s *= 2) blk.push_back((int32_t)s);
    std::vector<int> rounds;
    for (uint32_t rho = 0; rho < R; ++rho) {
        auto rows = b.zeros(), mask = b.zeros(), bias = b.zeros();
        for (uint32_t c = 0; c < C; ++c) {
            const uint32_t j = C * rho + c;
            if (j >= H) continue;
            for (int i = 0; i < d1.in_dim; ++i) rows[P * c + i] = d1.weight[(size_t)j * d1.in_dim + i];
            mask[P * c] = 1;
            bias[P * c] = bias_at(d1, (int)j);
        }
        int z = b.mulplain(0, b.cst(rows, true));
        z = b.rotate_and_sum(z, blk);
        z = b.mulplain(z, b.cst(mask, true), d1.bias ? b.cst(bias, false) : -1);
        rounds.push_back(z);
    }
    int h = b.combine_tree(rounds, 1);
    h = b.square(h);
    std::vector<int32_t> coll;
    for (uint32_t s = 1; s < next_pow2(std::max<uint32_t>(R, 2)); s *= 2) coll.push_back((int32_t)s);
    for (uint32_t s = P; s < N / 2 && s < P * C; s *= 2) coll.push_back((int32_t)s);
    if (P * C > N / 2) coll.push_back(LOLA_ROW_SWAP);
    p->output_map.assign((size_t)d2.out_dim * N, -1);
    for (int o = 0; o < d2.out_dim; ++o) {
        auto rows = b.zeros();
        for (uint32_t rho = 0; rho < R; ++rho)
            for (uint32_t c = 0; c < C; ++c) {
                const uint32_t j = C * rho + c;
                if (j < H) rows[P * c + rho] = d2.weight[(size_t)o * d2.in_dim + j];
            }
        int z = b.mulplain(h, b.cst(rows, true));
        z = b.rotate_and_sum(z, coll);
        if (d2.bias) {
            auto bv = b.zeros();
            bv[0] = d2.bias[o];
            z = b.addplain(z, b.cst(bv, false));
        }
        p->outputs.push_back(z);
        p->output_map[(size_t)o * N] = o;
    }
    return LOLA_OK;
}

// ---- cost model ---------------------------------------------------------
// Microseconds per operation of one request inside a large batch, measured on
// MI355X at N = 16384 with seven data primes (batched key switch 3.9, hoisted
// rotation 0.69 of that plus 0.48 of it once per source and wave, ct x ct
// product and relinearisation 24, plaintext product 0.55, one source of a
// linear combination 0.35, plaintext add 0.5); key switches and products
// scale with N log N and the number of limb transforms (L digit INTTs,
// dn (L+K) - L + 2K in the inner product, 2L in the mod-down: L^2 + 3L + 2
// with one special prime), element-wise passes with L N.
float predict_us(const lola_plan *p) {
    const double sN = (double)p->N / 16384.0, L = (double)p->L, K = (double)p->K;
    const double dn = std::ceil(L / K), M = L + K;
    const double ks = sN * (dn * M + 2 * K + 2 * L) / 72.0, ew = sN * L / 7.0;
    double us = 0;
    std::set<std::pair<int, int>> hoist_sources;   // (wave, source)
    for (const Op &o : p->ops) {
        if (o.kind == OP_ROT && o.hoist) {
            // hoisted: the gathered inner product and the mod-down, plus the
            // source's decomposition and transforms once per wave
            us += 3.9 * ks * 0.69;
            if (hoist_sources.insert({o.level, o.src}).second) us += 3.9 * ks * 0.48;
            continue;
        }
        switch (o.kind) {
            case OP_ROT:
            case OP_ROTADD: us += 3.9 * ks; break;
            case OP_SQUARE: us += 24.0 * ks; break;
            case OP_MULPLAIN: us += (0.55 + (o.cadd >= 0 ? 0.25 : 0.0)) * ew; break;
            case OP_LINCOMB: us += 0.35 * (double)o.srcs.size() * ew; break;
            case OP_ADDPLAIN: us += 0.5 * ew; break;
        }
    }
    return (float)us;
}

// Microseconds for one request alone: waves run one after another, and a
// wave's launches (linear combinations, plaintext ops, products with their
// relinearisation, key switches) one after another; a launch is priced by its
// rounds of workgroups over the 256 CUs.  Per round, measured on MI355X for
// single-request launches at N = 16384: one transform per workgroup (digits,
// mod-down, the key switch's latency form) 17-19 us, one transform plus its key
// products 13 us each in the batched inner stage (dn of them per workgroup),
// the exact product of a square 42 us at L = 7, a linear combination 12 us, a
// plaintext op 5 us.  Transform times scale with log2 N.  With K special
// primes a key switch has dn = ceil(L/K) digits and L + K target moduli.
float predict_latency_us(const lola_plan *p) {
    const double sl = std::log2((double)p->N) / 14.0, L = (double)p->L, K = (double)p->K;
    const double dn = std::ceil(L / K), M = L + K;
    auto rounds = [](double wgs) { return std::ceil(wgs / 256.0); };
    auto ks_us = [&](double n) {
        if (n <= 0) return 0.0;
        if (K == 1 && n * dn * M <= 256)   // terms straight from the input, then fold and mod-down together
            return 33.0 * sl + 34.0 * sl * rounds(2 * n * L);
        double t = 17.0 * sl * (rounds(n * L) + rounds(2 * n * L));   // digits, mod-down
        if (n <= 16) t += 19.0 * sl * (rounds(n * dn * M) + rounds(2 * n * M));   // terms, fold
        else t += 13.0 * sl * dn * rounds(n * M);
        return t;
    };
    double us = 0;
    for (uint32_t lev = 1; lev <= p->n_waves; ++lev) {
        double lin = 0, plain = 0, sq = 0, rot = 0, hrot = 0;
        std::set<int> hsrc;
        for (int i : p->level_ops[lev]) {
            if (p->ops[i].kind == OP_ROT && p->ops[i].hoist) {
                hrot += 1;
                hsrc.insert(p->ops[i].src);
                continue;
            }
            switch (p->ops[i].kind) {
                case OP_LINCOMB: lin += 1; break;
                case OP_MULPLAIN:
                case OP_ADDPLAIN: plain += 1; break;
                case OP_SQUARE: sq += 1; break;
                case OP_ROT:
                case OP_ROTADD: rot += 1; break;
            }
        }
        if (lin > 0) us += 12.0;
        if (plain > 0) us += 5.0;
        if (sq > 0) us += 42.0 * sl * (L / 7.0) * rounds(sq) + ks_us(sq);
        us += ks_us(rot);
        if (hrot > 0) {   // sources' digits and transforms, then gathered products and mod-down
            const double ns = (double)hsrc.size();
            us += 17.0 * sl * rounds(ns * L) + 19.0 * sl * rounds(ns * dn * M);
            // the gathered products read each rotation's key and its source's
            // transformed digits, 3 dn (L+K) limbs: many hoisted rotations in
            // a wave are bound by that traffic (about 5.5 TB/s measured)
            const double limb_bytes = 4.0 * (double)p->N;
            const double bytes_us = hrot * 3.0 * dn * M * limb_bytes / 5.5e6;
            us += std::max(14.0 * sl * (dn / 7.0) * rounds(hrot * (L + 2 * K)), bytes_us) + 17.0 * sl * rounds(2 * hrot * L);
        }
    }
    return (float)us;
}

// ---- levels and registers ---------------------------------------------
void schedule(lola_plan *p) {
    std::vector<int> level(p->n_regs, 0);
    auto srcs_of = [](const Op &o) {
        std::vector<int> s;
        if (o.kind == OP_LINCOMB) s = o.srcs;
        else s.push_back(o.src);
        if (o.kind == OP_ROTADD) s.push_back(o.addend);
        return s;
    };
    uint32_t maxl = 0;
    for (Op &o : p->ops) {
        int l = 0;
        for (int r : srcs_of(o)) l = std::max(l, level[r]);
        o.level = l + 1;
        level[o.dst] = o.level;
        maxl = std::max<uint32_t>(maxl, (uint32_t)o.level);
    }
    p->n_waves = maxl;
    p->level_ops.assign(maxl + 1, {});
    for (size_t i = 0; i < p->ops.size(); ++i) p->level_ops[p->ops[i].level].push_back((int)i);
    // last level at which each register is read
    std::vector<int> last(p->n_regs, -1);
    for (const Op &o : p->ops)
        for (int r : srcs_of(o)) last[r] = std::max(last[r], o.level);
    std::set<int> outs(p->outputs.begin(), p->outputs.end());
    p->phys.assign(p->n_regs, -1);
    std::vector<int> order(p->ops.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return p->ops[a].level < p->ops[c].level; });
    std::vector<int> free_list;
    std::vector<std::vector<int>> release(maxl + 2);
    for (uint32_t r = 0; r < p->n_regs; ++r)
        if (last[r] >= 0 && r >= p->n_inputs && !outs.count((int)r)) release[last[r]].push_back((int)r);
    uint32_t nphys = 0, cur_level = 0;
    std::vector<uint32_t> squares(maxl + 1, 0);
    std::vector<std::set<int>> hoist_src(maxl + 1);
    for (int idx : order) {
        const Op &o = p->ops[idx];
        while (cur_level < (uint32_t)o.level) {   // entering a new level: buffers last read earlier are free
            for (int r : release[cur_level]) free_list.push_back(p->phys[r]);
            ++cur_level;
        }
        if (o.kind == OP_SQUARE) squares[o.level]++;
        if (o.kind == OP_ROT && o.hoist) hoist_src[o.level].insert(o.src);
        if (outs.count(o.dst)) continue;
        if (free_list.empty()) free_list.push_back((int)nphys++);
        p->phys[o.dst] = free_list.back();
        free_list.pop_back();
    }
    p->n_phys = nphys;
    p->max_squares_per_wave = *std::max_element(squares.begin(), squares.end());
    p->max_hoist_per_wave = 0;
    for (const auto &hs : hoist_src) p->max_hoist_per_wave = std::max<uint32_t>(p->max_hoist_per_wave, (uint32_t)hs.size());
    std::set<uint32_t> g;
    for (const Op &o : p->ops)
        if (o.kind == OP_ROTADD || o.kind == OP_ROT) g.insert(o.galois);
    p->galois.assign(g.begin(), g.end());
}

}  // namespace
}  // namespace lola

using namespace lola;

extern "C" {

int compile_cifar_net(lola_plan *p, Builder &b, const lola_layer *ls, uint32_t n) {
    // CONV2D (C channels), SQUARE, CONV2D (over all maps), then SQUARE, DENSE
    // (one message per logit) or any other chain of DENSE and SQUARE layers,
    // continued from the second convolution's dense output with emit_chain
    if (n < 4 || ls[1].kind != LOLA_LAYER_SQUARE || ls[2].kind != LOLA_LAYER_CONV2D)
        return unsupported("two-convolution networks must be CONV2D, SQUARE, CONV2D, then DENSE and SQUARE layers");
    for (uint32_t l = 3; l < n; ++l)
        if (ls[l].kind != LOLA_LAYER_DENSE && ls[l].kind != LOLA_LAYER_SQUARE)
            return unsupported("two-convolution networks must be CONV2D, SQUARE, CONV2D, then DENSE and SQUARE layers");
    const bool classic = n == 5 && ls[3].kind == LOLA_LAYER_SQUARE && ls[4].kind == LOLA_LAYER_DENSE;
    const lola_layer &c1 = ls[0], &c2 = ls[2], &d = ls[classic ? 4 : 2];
    const uint32_t N = p->N;
    const int C = c1.in_dim > 0 ? c1.in_dim : 1;
    if (c1.in_h != c1.in_w || c1.k <= 0 || c1.stride <= 0 || c1.maps <= 0 || c1.in_h < c1.k || !c1.weight ||
        !c2.weight || c2.k <= 0 || c2.stride <= 0 || c2.maps <= 0)
        return unsupported("bad convolution shape");
    const int n1 = (c1.in_h - c1.k) / c1.stride + 1, V1 = n1 * n1, K = C * c1.k * c1.k;
    const int C2 = c2.in_dim > 0 ? c2.in_dim : 1;
    if (c2.in_h != n1 || c2.in_w != n1 || C2 != c1.maps || n1 < c2.k)
        return unsupported("second convolution must cover the first one's maps and outputs");
    const int n2 = (n1 - c2.k) / c2.stride + 1, V2 = n2 * n2, H = c2.maps * V2;
    if ((uint32_t)V1 > N / 2 || (uint32_t)H > N / 2) return unsupported("layer larger than a slot row");
    if (classic && (d.in_dim != H || !d.weight || d.out_dim <= 0))
        return unsupported("dense layer must take maps2*n2*n2 inputs");
    // inputs: convolution representation of every channel
    p->n_inputs = (uint32_t)K;
    p->queries = 1;
    p->n_regs = p->n_inputs;
    p->input_map.assign((size_t)K * N, -1);
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < c1.k; ++a)
            for (int e = 0; e < c1.k; ++e)
                for (int y = 0; y < n1; ++y)
                    for (int x = 0; x < n1; ++x)
                        p->input_map[(size_t)((c * c1.k + a) * c1.k + e) * N + y * n1 + x] =
                            (c * c1.in_h + c1.stride * y + a) * c1.in_w + c1.stride * x + e;
    // convolution 1: one linear combination of all K messages per map
    std::vector<int> ins(K);
    for (int i = 0; i < K; ++i) ins[i] = i;
    std::vector<int> maps;
    for (int m = 0; m < c1.maps; ++m) {
        std::vector<int64_t> w(c1.weight + (size_t)m * K, c1.weight + (size_t)(m + 1) * K);
        int cadd = -1;
        if (c1.bias) {
            auto v = b.zeros();
            for (int s = 0; s < V1; ++s) v[s] = c1.bias[m];
            cadd = b.cst(v, false);
        }
        maps.push_back(b.lincomb_any(ins, w, cadd));
    }
    // placement: R maps of V1 slots per slot row, 2R per message
    const uint32_t R = (N / 2) / (uint32_t)V1;
    const int G = (int)((c1.maps + 2 * R - 1) / (2 * R));
    std::vector<uint32_t> base(c1.maps);
    std::vector<int> msg(c1.maps);
    for (int m = 0; m < c1.maps; ++m) {
        msg[m] = m / (int)(2 * R);
        base[m] = ((uint32_t)m % (2 * R)) / R * (N / 2) + ((uint32_t)m % R) * (uint32_t)V1;
    }
    std::vector<int> sq;
    for (int g = 0; g < G; ++g) {
        std::vector<int> rows[2];
        for (int m = 0; m < c1.maps; ++m)
            if (msg[m] == g) rows[base[m] / (N / 2)].push_back(maps[m]);
        int y = b.combine_tree(rows[0], V1);
        if (!rows[1].empty()) y = b.rotadd(b.combine_tree(rows[1], V1), LOLA_ROW_SWAP, y);
        sq.push_back(b.square(y));
    }
    // convolution 2, dense vector - row major: one full-vector sum per output
    std::vector<int32_t> full;
    for (uint32_t s = 1; s < N / 2; s *= 2) full.push_back((int32_t)s);
    full.push_back(LOLA_ROW_SWAP);
    const int K2 = c2.k * c2.k;
    std::vector<int> gathered;
    auto bias2 = b.zeros();
    for (int j = 0; j < H; ++j) {
        const int mo = j / V2, y2 = (j % V2) / n2, x2 = j % n2;
        std::vector<int> parts;
        for (int g = 0; g < G; ++g) {
            auto row = b.zeros();
            for (int m = 0; m < c1.maps; ++m) {
                if (msg[m] != g) continue;
                for (int a = 0; a < c2.k; ++a)
                    for (int e = 0; e < c2.k; ++e)
                        row[base[m] + (uint32_t)(n1 * (c2.stride * y2 + a) + c2.stride * x2 + e)] =
                            c2.weight[((size_t)mo * c1.maps + m) * K2 + a * c2.k + e];
            }
            parts.push_back(b.mulplain(sq[g], b.cst(row, true)));
        }
        int z = parts.size() == 1 ? parts[0] : b.lincomb_any(parts, std::vector<int64_t>(parts.size(), 1), -1);
        z = b.rotate_and_sum(z, full);
        // the sparse outputs into one dense message: sparse vector - column
        // major with W = I (column j one-hot at slot j)
        auto onehot = b.zeros();
        onehot[j] = 1;
        gathered.push_back(b.column_term(z, std::move(onehot)));
        bias2[j] = bias_at(c2, mo);
    }
    // (+ all biases at once)
    int h = b.column_sum(gathered, c2.bias ? b.cst(bias2, false) : -1);
    if (!classic) {
        // a dense vector, value j at slot j
        ChainVec v;
        v.regs = {h};
        v.width = H;
        for (int j = 0; j < H; ++j) v.pos.push_back((uint32_t)j);
        const int rc = emit_chain(b, ls, 3, n, v);
        if (rc) return rc;
        chain_outputs(p, v);
        return LOLA_OK;
    }
    h = b.square(h);
    std::vector<int32_t> steps;
    for (uint32_t s = 1; s < next_pow2((uint32_t)H); s *= 2) steps.push_back((int32_t)s);
    if (steps.empty()) steps.push_back(1);
    p->output_map.assign((size_t)d.out_dim * N, -1);
    for (int o = 0; o < d.out_dim; ++o) {
        auto row = b.zeros();
        for (int i = 0; i < H; ++i) row[i] = d.weight[(size_t)o * H + i];
        int z = b.mulplain(h, b.cst(row, true));
        z = b.rotate_and_sum(z, steps);
        if (d.bias) {
            auto bv = b.zeros();
            bv[0] = d.bias[o];
            z = b.addplain(z, b.cst(bv, false));
        }
        p->outputs.push_back(z);
        p->output_map[(size_t)o * N] = o;
    }
    return LOLA_OK;
}

// Chains of DENSE and SQUARE layers on one query, each dense layer taking the
// recipe its input's representation calls for: sparse vector - column major
// on a sparse input (dense result, no rotation), dense vector - row major
// with a whole-message sum per row on a dense input (sparse result, one
// message per row); a square acts on every message.  sparse_input: the
// client sends value i as message i with v_i in every slot, so the first
// layer is column major (LOLA_RECIPE_SPARSE_COLUMN_MAJOR); otherwise one
// dense message, value i at slot i (LOLA_RECIPE_DENSE_CHAIN).
static bool is_dense_chain(const lola_layer *ls, uint32_t n) {
    if (n == 0 || ls[0].kind != LOLA_LAYER_DENSE) return false;
    for (uint32_t i = 0; i < n; ++i)
        if (ls[i].kind != LOLA_LAYER_DENSE && ls[i].kind != LOLA_LAYER_SQUARE) return false;
    return true;
}

int compile_dense_chain(lola_plan *p, Builder &b, const lola_layer *ls, uint32_t n, bool sparse_input) {
    const uint32_t N = p->N;
    if (!is_dense_chain(ls, n)) return unsupported("a dense chain holds DENSE and SQUARE layers, DENSE first");
    const int k = ls[0].in_dim;
    if (k <= 0 || (uint32_t)k > N) return unsupported("dense layer larger than a message");
    p->queries = 1;
    ChainVec v;
    v.width = k;
    v.sparse = sparse_input;
    if (sparse_input) {
        p->n_inputs = (uint32_t)k;
        p->input_map.assign((size_t)k * N, -1);
        for (int i = 0; i < k; ++i) {
            std::fill(p->input_map.begin() + (size_t)i * N, p->input_map.begin() + (size_t)(i + 1) * N, i);
            v.regs.push_back(i);
        }
    } else {
        p->n_inputs = 1;
        p->input_map.assign(N, -1);
        for (int i = 0; i < k; ++i) {
            p->input_map[i] = i;
            v.pos.push_back((uint32_t)i);
        }
        v.regs.push_back(0);
    }
    p->n_regs = p->n_inputs;
    const int rc = emit_chain(b, ls, 0, n, v);
    if (rc) return rc;
    chain_outputs(p, v);
    p->recipe = sparse_input ? LOLA_RECIPE_SPARSE_COLUMN_MAJOR : LOLA_RECIPE_DENSE_CHAIN;
    return LOLA_OK;
}

// The recipes that apply to a layer list: DENSE, SQUARE, DENSE has two for
// its dense layers, convolution networks with layers after the first dense
// one two for that layer's reduction; everything else has one
// (LOLA_RECIPE_FIXED).
// The dense-chain recipes take any chain of DENSE and SQUARE layers and are
// the candidates for chains that no other pattern covers; they can be forced
// on the others.
static bool dense_pattern(const lola_layer *layers, uint32_t n_layers) {
    const lola_layer &l0 = layers[0];
    if (l0.kind != LOLA_LAYER_DENSE) return false;
    if (n_layers == 3 && layers[1].kind == LOLA_LAYER_SQUARE && layers[2].kind == LOLA_LAYER_DENSE) return true;
    return n_layers == 1 || (n_layers == 2 && layers[1].kind == LOLA_LAYER_SQUARE);
}
static std::vector<int> recipe_candidates(const lola_layer *layers, uint32_t n_layers) {
    const lola_layer &l0 = layers[0];
    if (l0.kind == LOLA_LAYER_DENSE && n_layers == 3 && dense_pattern(layers, n_layers))
        return {LOLA_RECIPE_DENSE_ROW_MAJOR, LOLA_RECIPE_STACKED_ROW_MAJOR};
    if ((l0.kind == LOLA_LAYER_CONV2D || l0.kind == LOLA_LAYER_CONV2D_DENSE_INPUT) && n_layers >= 4 &&
        layers[2].kind != LOLA_LAYER_CONV2D)
        return {LOLA_RECIPE_FULL_REDUCTION, LOLA_RECIPE_SHARED_REDUCTION};
    if (is_dense_chain(layers, n_layers) && !dense_pattern(layers, n_layers))
        return {LOLA_RECIPE_DENSE_CHAIN, LOLA_RECIPE_SPARSE_COLUMN_MAJOR};
    return {LOLA_RECIPE_FIXED};
}
static bool recipe_applies(const lola_layer *layers, uint32_t n_layers, int recipe) {
    if ((recipe == LOLA_RECIPE_DENSE_CHAIN || recipe == LOLA_RECIPE_SPARSE_COLUMN_MAJOR) &&
        is_dense_chain(layers, n_layers))
        return true;
    const std::vector<int> cand = recipe_candidates(layers, n_layers);
    return std::find(cand.begin(), cand.end(), recipe) != cand.end();
}

// Compiles with one recipe (one of recipe_candidates()).
static int compile_with(const lola_params *prm, const lola_layer *layers, uint32_t n_layers, int recipe,
                        int sums, lola_plan **out) {
    *out = nullptr;
    lola_plan *p = new lola_plan();
    p->N = prm->N;
    p->L = prm->L;
    p->K = prm->P2 ? 2u : 1u;
    p->t = prm->t;
    p->sums = (uint32_t)sums;
    Builder b{p};
    b.hoist_sums = sums == LOLA_SUMS_HOISTED;
    int rc;
    const lola_layer &l0 = layers[0];
    const uint32_t N = prm->N;
    const bool head = l0.kind == LOLA_LAYER_DENSE && n_layers == 3;
    if (recipe == LOLA_RECIPE_DENSE_CHAIN || recipe == LOLA_RECIPE_SPARSE_COLUMN_MAJOR) {
        rc = compile_dense_chain(p, b, layers, n_layers, recipe == LOLA_RECIPE_SPARSE_COLUMN_MAJOR);
    } else if (l0.kind == LOLA_LAYER_CONV2D && n_layers >= 4 && layers[2].kind == LOLA_LAYER_CONV2D) {
        rc = compile_cifar_net(p, b, layers, n_layers);
    } else if (l0.kind == LOLA_LAYER_CONV2D || l0.kind == LOLA_LAYER_CONV2D_DENSE_INPUT) {
        rc = compile_conv_net(p, b, layers, n_layers, recipe == LOLA_RECIPE_SHARED_REDUCTION);
    } else if (l0.kind == LOLA_LAYER_DENSE && l0.weight && l0.in_dim > 0 && l0.out_dim > 0) {
        if ((uint32_t)l0.in_dim > N / 2) {
            rc = unsupported("dense input longer than a slot row");
        } else if (head) {
            if (recipe == LOLA_RECIPE_STACKED_ROW_MAJOR) {
                rc = compile_dense_head_stacked(p, b, layers, n_layers);
                p->recipe = LOLA_RECIPE_STACKED_ROW_MAJOR;
            } else {
                rc = compile_dense_head(p, b, layers, n_layers);
                p->recipe = LOLA_RECIPE_DENSE_ROW_MAJOR;
            }
        } else if ((uint32_t)l0.in_dim <= N / 4) {
            rc = compile_stacked_dense(p, b, layers, n_layers);
        } else {
            rc = unsupported("a single dense layer needs in_dim <= N/4 (stacked input)");
        }
    } else {
        rc = unsupported("first layer must be CONV2D or DENSE");
    }
    if (rc) {
        delete p;
        return rc;
    }
    schedule(p);
    p->predicted_us = predict_us(p);
    p->predicted_latency_us = predict_latency_us(p);
    *out = p;
    return LOLA_OK;
}

int lola_compile_ex(const lola_params *prm, const lola_layer *layers, uint32_t n_layers,
                    const lola_compile_options *opts, lola_plan **out) {
    if (!prm || !layers || !out || n_layers == 0) return set_error(LOLA_E_INVAL, "null argument");
    *out = nullptr;
    if (prm->N < 1024 || prm->N > 16384 || (prm->N & (prm->N - 1)) || prm->t < 3 || prm->L < 1)
        return set_error(LOLA_E_PARAMS, "bad N, t or L");
    const int objective = opts ? opts->objective : LOLA_OBJECTIVE_THROUGHPUT;
    const int recipe = opts ? opts->recipe : LOLA_RECIPE_AUTO;
    const int sums = opts ? opts->sums : LOLA_SUMS_AUTO;
    if (objective != LOLA_OBJECTIVE_THROUGHPUT && objective != LOLA_OBJECTIVE_LATENCY)
        return set_error(LOLA_E_INVAL, "unknown objective");
    if (recipe < LOLA_RECIPE_AUTO || recipe > LOLA_RECIPE_SPARSE_COLUMN_MAJOR)
        return set_error(LOLA_E_INVAL, "unknown recipe");
    if (sums < LOLA_SUMS_AUTO || sums > LOLA_SUMS_HOISTED) return set_error(LOLA_E_INVAL, "unknown sums form");
    // sums forms to build: the one asked for; by default the sequential form,
    // and for the latency objective the hoisted one beside it
    std::vector<int> forms;
    if (sums != LOLA_SUMS_AUTO) forms = {sums};
    else if (objective == LOLA_OBJECTIVE_LATENCY) forms = {LOLA_SUMS_SEQUENTIAL, LOLA_SUMS_HOISTED};
    else forms = {LOLA_SUMS_SEQUENTIAL};
    std::vector<int> cand = recipe_candidates(layers, n_layers);
    if (recipe != LOLA_RECIPE_AUTO) {
        if (!recipe_applies(layers, n_layers, recipe))
            return unsupported("the recipe does not apply to this layer list");
        cand = {recipe};
    }
    // every candidate; keep the cheapest for the objective (the first on ties)
    auto cost = [&](const lola_plan *q) {
        return objective == LOLA_OBJECTIVE_LATENCY ? q->predicted_latency_us : q->predicted_us / (float)q->queries;
    };
    lola_plan *best = nullptr;
    int first_rc = LOLA_OK;
    for (int f : forms)
        for (int r : cand) {
            lola_plan *q = nullptr;
            const int rc = compile_with(prm, layers, n_layers, r, f, &q);
            if (rc) {
                if (!first_rc) first_rc = rc;
                continue;
            }
            if (!best || cost(q) < cost(best)) {
                delete best;
                best = q;
            } else {
                delete q;
            }
        }
    if (!best) return first_rc;
    *out = best;
    return LOLA_OK;
}

int lola_compile(const lola_params *prm, const lola_layer *layers, uint32_t n_layers, lola_plan **out) {
    return lola_compile_ex(prm, layers, n_layers, nullptr, out);
}

int lola_plan_get_info(const lola_plan *p, lola_plan_info *info) {
    if (!p || !info) return set_error(LOLA_E_INVAL, "null argument");
    memset(info, 0, sizeof *info);
    info->n_inputs = p->n_inputs;
    info->n_outputs = (uint32_t)p->outputs.size();
    info->n_ops = (uint32_t)p->ops.size();
    info->n_consts = (uint32_t)p->consts.size();
    info->n_galois = (uint32_t)p->galois.size();
    info->n_waves = p->n_waves;
    info->queries = p->queries;
    info->n_phys_regs = p->n_phys;
    info->recipe = p->recipe;
    info->predicted_us = p->predicted_us;
    info->predicted_latency_us = p->predicted_latency_us;
    info->sums = p->sums;
    for (const Op &o : p->ops) {
        switch (o.kind) {
            case OP_LINCOMB:
                info->n_mul_scalar += (uint32_t)o.srcs.size();
                info->n_add += (uint32_t)o.srcs.size() - 1;
                if (o.cadd >= 0) info->n_add_plain++;
                break;
            case OP_MULPLAIN:
                info->n_mul_plain++;
                if (o.cadd >= 0) info->n_add_plain++;
                break;
            case OP_ADDPLAIN: info->n_add_plain++; break;
            case OP_ROTADD: info->n_rotations++; info->n_add++; break;
            case OP_ROT: info->n_rotations++; break;
            case OP_SQUARE: info->n_square++; break;
        }
    }
    return LOLA_OK;
}

int lola_plan_galois(const lola_plan *p, uint32_t *g) {
    if (!p || !g) return set_error(LOLA_E_INVAL, "null argument");
    std::copy(p->galois.begin(), p->galois.end(), g);
    return LOLA_OK;
}

int lola_plan_input_map(const lola_plan *p, int32_t *m) {
    if (!p || !m) return set_error(LOLA_E_INVAL, "null argument");
    std::copy(p->input_map.begin(), p->input_map.end(), m);
    return LOLA_OK;
}

int lola_plan_output_map(const lola_plan *p, int32_t *m) {
    if (!p || !m) return set_error(LOLA_E_INVAL, "null argument");
    std::copy(p->output_map.begin(), p->output_map.end(), m);
    return LOLA_OK;
}

int lola_plan_dump(const lola_plan *p, char *buf, size_t cap) {
    if (!p) return set_error(LOLA_E_INVAL, "null argument");
    std::string s;
    auto step = [](int32_t k) { return k == LOLA_ROW_SWAP ? std::string("swap") : std::to_string(k); };
    for (const Op &o : p->ops) {
        switch (o.kind) {
            case OP_LINCOMB:
                s += "lincomb " + std::to_string(o.dst);
                for (size_t k = 0; k < o.srcs.size(); ++k)
                    s += " " + std::to_string(o.srcs[k]) + ":" + std::to_string(o.w[k]);
                if (o.cadd >= 0) s += " +add " + std::to_string(o.cadd);
                break;
            case OP_MULPLAIN:
                s += "mulplain " + std::to_string(o.dst) + " " + std::to_string(o.src) + " " + std::to_string(o.cmul);
                if (o.cadd >= 0) s += " +add " + std::to_string(o.cadd);
                break;
            case OP_ADDPLAIN:
                s += "addplain " + std::to_string(o.dst) + " " + std::to_string(o.src) + " " + std::to_string(o.cadd);
                break;
            case OP_ROTADD:
                s += "rotadd " + std::to_string(o.dst) + " " + std::to_string(o.src) + " " + step(o.step) + " " +
                     std::to_string(o.addend);
                break;
            case OP_ROT:
                s += (o.hoist ? "hrot " : "rot ") + std::to_string(o.dst) + " " + std::to_string(o.src) + " " +
                     step(o.step);
                break;
            case OP_SQUARE: s += "square " + std::to_string(o.dst) + " " + std::to_string(o.src); break;
        }
        s += "\n";
    }
    s += "outputs";
    for (int r : p->outputs) s += " " + std::to_string(r);
    s += "\n";
    if (!buf || cap < s.size() + 1) return (int)(s.size() + 1);
    memcpy(buf, s.c_str(), s.size() + 1);
    return LOLA_OK;
}

int lola_plan_const(const lola_plan *p, uint32_t id, int64_t *slots) {
    if (!p || !slots) return set_error(LOLA_E_INVAL, "null argument");
    if (id >= p->consts.size()) return set_error(LOLA_E_INVAL, "constant id out of range");
    std::copy(p->consts[id].begin(), p->consts[id].end(), slots);
    return LOLA_OK;
}

}  // extern "C"
