// A launch program: a blob of job descriptors plus the ordered list of
// batched launches that read them.  Building a program assigns scratch
// regions and writes every descriptor on the host; running it only issues
// kernel launches with device pointers into the uploaded blob, so a run can
// be captured in a HIP graph and replayed.
#pragma once
#include <cstring>

#include "lola_internal.hpp"

namespace lola {

// Element-wise jobs (one ciphertext each, 2 L N words).
constexpr uint32_t LIN_MAX = 32;   // sources of one linear combination
constexpr uint32_t LIN_OUT = 8;    // outputs of one job (combinations of the same sources)
struct LinJob {              // dst[d] = sum_k w[d]_k src_k (+ add-form constant add[d] on c0), d < n_dst
    const uint32_t *srcs[LIN_MAX];
    const uint32_t *w[LIN_OUT];    // device [n_src][2][L]: residue, Montgomery form (w 2^32 mod q) per limb
    const uint32_t *add[LIN_OUT];  // [L][N] add-form constant or null
    uint32_t *dst[LIN_OUT];
    uint32_t n_src, n_dst;
};

// Merges single-output jobs whose source lists are equal (the maps of a
// convolution over the same input messages) into jobs of up to LIN_OUT
// outputs, so each source is read once for all of them.  Order within a
// launch does not matter: the jobs of one level are independent.
inline std::vector<LinJob> group_lincombs(const std::vector<LinJob> &single) {
    std::vector<LinJob> out;
    std::vector<size_t> open;   // indices in out of groups that still take outputs
    for (const LinJob &j : single) {
        size_t g = out.size();
        for (size_t k : open) {
            const LinJob &c = out[k];
            if (c.n_dst < LIN_OUT && c.n_src == j.n_src &&
                std::equal(j.srcs, j.srcs + j.n_src, c.srcs)) {
                g = k;
                break;
            }
        }
        if (g == out.size()) {
            out.push_back(j);
            open.push_back(g);
            continue;
        }
        LinJob &c = out[g];
        for (uint32_t d = 0; d < j.n_dst && c.n_dst < LIN_OUT; ++d) {
            c.w[c.n_dst] = j.w[d];
            c.add[c.n_dst] = j.add[d];
            c.dst[c.n_dst] = j.dst[d];
            ++c.n_dst;
        }
        if (c.n_dst == LIN_OUT) open.erase(std::find(open.begin(), open.end(), g));
    }
    return out;
}
struct PlainJob {            // dst = src * mul (+ add on c0); mul or add may be null
    const uint32_t *src;
    const uint32_t *mul;     // [L][N] Montgomery mul-form constant
    const uint32_t *add;     // [L][N] add-form constant
    uint32_t *dst;
};
struct MulJob {
    const uint32_t *a, *b;   // [2][L][N] NTT form
    uint32_t *out3;          // [3][L][N] NTT form
    uint32_t *scr;           // mul_scratch_words words
};

enum LaunchKind : uint32_t {
    LK_NTT, LK_LIN, LK_PLAIN, LK_KS, LK_MUL_EXTEND, LK_MUL_PRODUCT, LK_MUL_ROUND,
    LK_KS_HSRC,   // hoisted rotations: decomposition and transforms of each source
    LK_KS_HROT    // hoisted rotations: gathered inner products and mod-down
};
struct Launch {
    uint32_t kind, n;
    size_t off;              // byte offset of the descriptors in the blob
    uint64_t aux[6] = {0, 0, 0, 0, 0, 0};   // job counts for the algorithmic cost (launch_aux)
};

// What a launch's algorithmic cost depends on beyond its job count.  Bytes
// count each distinct buffer a launch reads once (jobs of a batch share
// sources, constants and keys, read from HBM once and then from cache);
// lane-ops count every job's work.
//   LinJob:   source-output terms, distinct sources, outputs with a constant,
//             distinct constants, outputs
//   PlainJob: jobs with a product, distinct product constants, jobs with an add, distinct add constants
//   MulJob:   squares (a == b: one operand extended and read)
//   KsJob:    distinct keys, distinct hoisting sources
template <class T, class F>
inline uint64_t n_distinct(const std::vector<T> &v, F key) {
    std::vector<const void *> k;
    for (const T &j : v)
        if (key(j)) k.push_back(key(j));
    std::sort(k.begin(), k.end());
    return (uint64_t)(std::unique(k.begin(), k.end()) - k.begin());
}
inline void launch_aux(const std::vector<LinJob> &v, uint64_t *a) {
    std::vector<const void *> src, add;
    for (const LinJob &j : v) {
        a[0] += (uint64_t)j.n_src * j.n_dst;
        a[4] += j.n_dst;
        src.insert(src.end(), j.srcs, j.srcs + j.n_src);
        for (uint32_t d = 0; d < j.n_dst; ++d)
            if (j.add[d]) {
                ++a[2];
                add.push_back(j.add[d]);
            }
    }
    std::sort(src.begin(), src.end());
    a[1] = (uint64_t)(std::unique(src.begin(), src.end()) - src.begin());
    std::sort(add.begin(), add.end());
    a[3] = (uint64_t)(std::unique(add.begin(), add.end()) - add.begin());
}
inline void launch_aux(const std::vector<PlainJob> &v, uint64_t *a) {
    for (const PlainJob &j : v) {
        a[0] += j.mul != nullptr;
        a[2] += j.add != nullptr;
    }
    a[1] = n_distinct(v, [](const PlainJob &j) { return (const void *)j.mul; });
    a[3] = n_distinct(v, [](const PlainJob &j) { return (const void *)j.add; });
}
inline void launch_aux(const std::vector<MulJob> &v, uint64_t *a) {
    for (const MulJob &j : v) a[0] += j.a == j.b;
}
inline void launch_aux(const std::vector<KsJob> &v, uint64_t *a) {
    a[0] = n_distinct(v, [](const KsJob &j) { return (const void *)j.key; });
    a[1] = n_distinct(v, [](const KsJob &j) { return (const void *)j.hoist; });
}
template <class T>
inline void launch_aux(const std::vector<T> &, uint64_t *) {}

struct Program {
    std::vector<uint8_t> blob;
    std::vector<Launch> launches;
    size_t ks_jobs = 0;      // key switches issued (for reporting)

    size_t reserve_bytes(size_t bytes) {
        size_t off = (blob.size() + 255) & ~(size_t)255;
        blob.resize(off + bytes);
        return off;
    }
    template <class T>
    size_t put(const std::vector<T> &v) {
        size_t off = reserve_bytes(v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
    template <class T>
    void launch(LaunchKind k, const std::vector<T> &v) {
        if (v.empty()) return;
        Launch l{(uint32_t)k, (uint32_t)v.size(), put(v)};
        launch_aux(v, l.aux);
        launches.push_back(l);
    }
};

// Appends src's descriptors and launches to dst (offsets moved to where the
// descriptors land in dst's blob).
inline void append_program(Program &dst, const Program &src) {
    if (src.blob.empty()) return;
    const size_t base = dst.reserve_bytes(src.blob.size());
    std::memcpy(dst.blob.data() + base, src.blob.data(), src.blob.size());
    for (Launch l : src.launches) {
        l.off += base;
        dst.launches.push_back(l);
    }
    dst.ks_jobs += src.ks_jobs;
}

// Builders.  Key switches and products are split into chunks that reuse the
// scratch region [scratch, scratch + chunk * per-job words) in stream order.
void program_keyswitch(const lola_ctx *ctx, Program &p, std::vector<KsJob> jobs, uint32_t *scratch,
                       uint32_t chunk, LaunchKind kind = LK_KS);
void program_mul(const lola_ctx *ctx, Program &p, const std::vector<MulJob> &pairs, uint32_t *scratch,
                 uint32_t chunk);

// Issues the launches; d_blob is the device copy of p.blob.
int program_run(lola_ctx *ctx, const Program &p, const uint8_t *d_blob, hipStream_t s);
// Issues one launch of a program.
int program_run_launch(lola_ctx *ctx, const Launch &l, const uint8_t *d_blob, hipStream_t s);
// Uploads the blob through the context's descriptor ring and runs (immediate
// API calls; the blob must fit one ring slab).
int program_run_now(lola_ctx *ctx, const Program &p, hipStream_t s);

// Kernel launchers on device descriptor arrays.
int launch_lin_dev(lola_ctx *ctx, const LinJob *d, uint32_t n, const uint64_t *aux, hipStream_t s);
int launch_plain_dev(lola_ctx *ctx, const PlainJob *d, uint32_t n, const uint64_t *aux, hipStream_t s);
int launch_keyswitch(lola_ctx *ctx, const KsJob *d, uint32_t n, const uint64_t *aux, hipStream_t s);
// Hoisted rotations: sources (x = c1, scratch = hoist area, galois 1), then
// rotations (hoist = the source's area, scratch = their own).
int launch_keyswitch_hoist_src(lola_ctx *ctx, const KsJob *d, uint32_t n, hipStream_t s);
int launch_keyswitch_hoist_rot(lola_ctx *ctx, const KsJob *d, uint32_t n, const uint64_t *aux, hipStream_t s);
int launch_mul_stage(lola_ctx *ctx, uint32_t stage, const MulJob *d, uint32_t n, uint64_t n_squares, hipStream_t s);

}  // namespace lola
