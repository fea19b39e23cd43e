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
struct LinJob {              // dst = sum_k w_k src_k (+ add-form constant on c0)
    const uint32_t *srcs[LIN_MAX];
    const uint32_t *w;             // device [n_src][2][L]: residue, Shoup companion per limb
    const uint32_t *add;           // [L][N] add-form constant or null
    uint32_t *dst;
    uint32_t n_src, pad;
};
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
};

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
        launches.push_back(Launch{(uint32_t)k, (uint32_t)v.size(), put(v)});
    }
};

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
int launch_lin_dev(lola_ctx *ctx, const LinJob *d, uint32_t n, hipStream_t s);
int launch_plain_dev(lola_ctx *ctx, const PlainJob *d, uint32_t n, hipStream_t s);
int launch_keyswitch(lola_ctx *ctx, const KsJob *d, uint32_t n, hipStream_t s);
// Hoisted rotations: sources (x = c1, scratch = hoist area, galois 1), then
// rotations (hoist = the source's area, scratch = their own).
int launch_keyswitch_hoist_src(lola_ctx *ctx, const KsJob *d, uint32_t n, hipStream_t s);
int launch_keyswitch_hoist_rot(lola_ctx *ctx, const KsJob *d, uint32_t n, hipStream_t s);
int launch_mul_stage(lola_ctx *ctx, uint32_t stage, const MulJob *d, uint32_t n, hipStream_t s);

}  // namespace lola
