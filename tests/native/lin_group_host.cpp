// Host check of the grouping of linear combinations into multi-output jobs
// (group_lincombs) and of the launch cost counts of linear-combination
// launches (launch_aux): jobs whose source lists are equal merge, up to
// LIN_OUT outputs each, every output keeps its own weights, constant and
// destination exactly once, and jobs with different sources never merge.
// Pointers are tags only (never dereferenced).  Exit status = failures.
#include "../../paper_1812_10659_amd/csrc/program.hpp"

#include <cstdio>
#include <map>
#include <set>

using namespace lola;

static const uint32_t *tag(uintptr_t v) { return reinterpret_cast<const uint32_t *>(v * 64); }

int main() {
    int fail = 0;
    std::vector<LinJob> single;
    // 3 source lists: A (25 sources, 13 outputs), B (25 other sources, 3
    // outputs), C (a prefix of A, 5 outputs: must not merge with A)
    auto add_job = [&](int list, int k, uintptr_t out_id) {
        LinJob j{};
        const int n = list == 2 ? 20 : 25;
        for (int s = 0; s < n; ++s) j.srcs[s] = tag(list == 1 ? 1000 + s : 1 + s);
        j.n_src = n;
        j.n_dst = 1;
        j.w[0] = tag(5000 + out_id);
        j.add[0] = (k % 2) ? tag(9000 + out_id) : nullptr;
        j.dst[0] = const_cast<uint32_t *>(tag(7000 + out_id));
        single.push_back(j);
    };
    uintptr_t id = 0;
    for (int k = 0; k < 13; ++k) add_job(0, k, id++);
    for (int k = 0; k < 3; ++k) add_job(1, k, id++);
    for (int k = 0; k < 5; ++k) add_job(2, k, id++);
    add_job(0, 1, id++);   // one more for list A after others
    const std::vector<LinJob> g = group_lincombs(single);
    std::map<const uint32_t *, int> seen;
    size_t outs = 0;
    for (const LinJob &j : g) {
        if (j.n_dst == 0 || j.n_dst > LIN_OUT) ++fail;
        for (uint32_t d = 0; d < j.n_dst; ++d) {
            const uintptr_t o = reinterpret_cast<uintptr_t>(j.dst[d]) / 64 - 7000;
            if (reinterpret_cast<uintptr_t>(j.w[d]) / 64 != 5000 + o) ++fail;
            const bool has_add = j.add[d] != nullptr;
            if (has_add && reinterpret_cast<uintptr_t>(j.add[d]) / 64 != 9000 + o) ++fail;
            ++seen[j.dst[d]];
            ++outs;
        }
        // every output's source list must be this job's
        for (const LinJob &s : single)
            for (uint32_t d = 0; d < j.n_dst; ++d)
                if (s.dst[0] == j.dst[d] &&
                    (s.n_src != j.n_src || !std::equal(s.srcs, s.srcs + s.n_src, j.srcs)))
                    ++fail;
    }
    if (outs != single.size() || seen.size() != single.size()) ++fail;
    for (auto &kv : seen)
        if (kv.second != 1) ++fail;
    // A: 14 outputs -> 2 jobs; B: 3 -> 1; C: 5 -> 1
    if (g.size() != 4) ++fail;
    uint64_t a[6] = {0, 0, 0, 0, 0, 0};
    launch_aux(g, a);
    const uint64_t terms = 14 * 25 + 3 * 25 + 5 * 20;
    if (a[0] != terms || a[1] != 25 + 25 || a[4] != single.size()) ++fail;
    uint64_t with_add = 0;
    for (const LinJob &s : single) with_add += s.add[0] != nullptr;
    if (a[2] != with_add || a[3] != with_add) ++fail;
    std::printf("lin grouping: %s (%zu jobs)\n", fail ? "FAILED" : "ok", g.size());
    return fail;
}
