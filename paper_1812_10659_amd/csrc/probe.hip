// VALU issue-rate probe: the rate at which the GPU retires the 32-bit
// integer instructions the modular arithmetic is built from, to state the
// peak the kernels are measured against (lane-ops per second).
//
// Each thread runs eight independent chains of one instruction kind, so the
// rate is bound by issue, not by an instruction's latency; the chains'
// values are written out so that no work is dropped.  Grid: 8 workgroups of
// 256 threads per compute unit.
#include "lola_internal.hpp"

namespace lola {

constexpr uint32_t PROBE_CHAINS = 8, PROBE_UNROLL = 16;

// Each step is one instruction written out (so the compiler can neither fold
// nor fuse the chains): OP 0 v_mul_lo_u32, 1 v_mul_hi_u32, 2 v_add_u32.
template <int OP>
__global__ __launch_bounds__(256) void valu_probe_kernel(uint32_t iters, uint32_t y, uint32_t *__restrict__ out) {
    uint32_t x[PROBE_CHAINS];
#pragma unroll
    for (uint32_t c = 0; c < PROBE_CHAINS; ++c) x[c] = threadIdx.x * 2654435761u + c * 40503u + blockIdx.x;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (uint32_t u = 0; u < PROBE_UNROLL; ++u) {
#pragma unroll
            for (uint32_t c = 0; c < PROBE_CHAINS; ++c) {
                if (OP == 0) {
                    asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[c]) : "v"(y));
                } else if (OP == 1) {
                    asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[c]) : "v"(y));
                } else {
                    asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[c]) : "v"(y));
                }
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (uint32_t c = 0; c < PROBE_CHAINS; ++c) r ^= x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

}  // namespace lola

using namespace lola;

extern "C" {

int lola_valu_probe(int op, uint32_t iters, uint32_t *out_dev, uint32_t out_words, double *lane_ops_per_s,
                    lola_stream stream) {
    if (!out_dev || !lane_ops_per_s || op < 0 || op > 2 || iters == 0) return set_error(LOLA_E_INVAL, "bad argument");
    int dev = 0, cus = 0;
    LOLA_HIP(hipGetDevice(&dev));
    LOLA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const uint32_t blocks = 8u * (uint32_t)cus, threads = 256;
    if ((size_t)out_words < (size_t)blocks * threads) return set_error(LOLA_E_SHAPE, "output buffer too small");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a = nullptr, b = nullptr;
    LOLA_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return set_error(LOLA_E_DEVICE, "event");
    }
    int rc = LOLA_OK;
    const uint32_t y = 0x9E3779B1u;
    auto launch = [&](uint32_t n) {
        if (op == 0) hipLaunchKernelGGL(valu_probe_kernel<0>, dim3(blocks), dim3(threads), 0, s, n, y, out_dev);
        else if (op == 1) hipLaunchKernelGGL(valu_probe_kernel<1>, dim3(blocks), dim3(threads), 0, s, n, y, out_dev);
        else hipLaunchKernelGGL(valu_probe_kernel<2>, dim3(blocks), dim3(threads), 0, s, n, y, out_dev);
    };
    launch(1);   // warm up
    float ms = 0;
    if (hipEventRecord(a, s) != hipSuccess) rc = set_error(LOLA_E_DEVICE, "event");
    if (!rc) launch(iters);
    if (!rc && (hipGetLastError() != hipSuccess || hipEventRecord(b, s) != hipSuccess ||
                hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
        rc = set_error(LOLA_E_DEVICE, "probe launch");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    const double ops = (double)blocks * threads * iters * PROBE_UNROLL * PROBE_CHAINS;
    *lane_ops_per_s = ms > 0 ? ops / (ms * 1e-3) : 0.0;
    return LOLA_OK;
}

}  // extern "C"
