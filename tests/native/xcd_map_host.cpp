// Host check of the key-switch kernels' block -> (job, unit) mappings: over
// the grid xcd_grid(n, units), every (job, unit) with job < n is produced by
// exactly one block; blocks past the last job map to job >= n; every block on
// XCD x takes a job of that XCD's contiguous range; and with lead long units
// per job, each XCD's blocks (in dispatch order) hand out all of its jobs'
// long units before any short one.  Exit status = number of failures.
#include "../../paper_1812_10659_amd/csrc/ks_core.hpp"

#include <cstdio>
#include <vector>

using namespace lola;

static int check(uint32_t n, uint32_t units, uint32_t lead) {
    const uint32_t grid = xcd_grid(n, units), per_xcd = (n + N_XCD - 1) / N_XCD;
    std::vector<int> seen((size_t)n * units, 0);
    std::vector<int> short_seen(N_XCD, 0);
    int bad = 0;
    for (uint32_t k = 0; k < grid; ++k) {
        const JobUnit ju = lead ? xcd_job_unit_lead(k, units, lead, n) : xcd_job_unit(k, units, n);
        const uint32_t x = k % N_XCD;
        if (ju.unit >= units) ++bad;
        if (ju.job / per_xcd != x && ju.job < per_xcd * N_XCD) ++bad;
        if (ju.job >= n) continue;
        ++seen[(size_t)ju.job * units + ju.unit];
        if (lead) {
            if (ju.unit >= lead) short_seen[x] = 1;
            else if (short_seen[x]) ++bad;   // a long unit after a short one on this XCD
        }
    }
    for (int c : seen)
        if (c != 1) ++bad;
    if (bad) std::printf("n=%u units=%u lead=%u: %d failures\n", n, units, lead, bad);
    return bad;
}

int main() {
    int bad = 0, cases = 0;
    for (uint32_t n = 1; n <= 260; ++n)
        for (uint32_t L = 1; L <= 12; ++L) {
            bad += check(n, L + 1, 0) + check(n, L + 1, 1) + check(n, L + 2, 2) + check(n, 2 * L, 0);
            cases += 4;
        }
    std::printf("%s (%d cases)\n", bad ? "FAILED" : "ok", cases);
    return bad ? 1 : 0;
}
