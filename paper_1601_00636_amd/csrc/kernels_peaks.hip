// Throughput probes for the roofline of the sweep: the integer VALU rate of
// v_bcnt_u32_b32 (popcount with accumulate, the sweep's most frequent
// instruction) and the LDS read bandwidth of conflict-free 64-bit reads, both
// measured on the running device rather than taken from its data sheet.
#include "internal.h"

namespace cuboid {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kChains = 8;           // independent dependency chains per lane
constexpr int kLdsWords = 4096;      // 32 KiB of LDS per workgroup

// kChains chains of x <- popcount(x) + x: one v_bcnt_u32_b32 per step, no
// two steps of a chain independent, so the compiler cannot fold the loop.
__global__ void __launch_bounds__(kProbeThreads) valu_probe_kernel(uint32_t iters, uint32_t *out) {
    uint32_t x[kChains];
    for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 131u + c * 7919u + blockIdx.x;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_popcount(x[c]) + x[c];
    }
    uint32_t s = 0;
    for (int c = 0; c < kChains; ++c) s ^= x[c];
    out[blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// Lane-linear 64-bit reads (consecutive lanes, consecutive words: no bank
// conflicts), 16 per step at constant offsets, folded into two accumulators.
__global__ void __launch_bounds__(kProbeThreads) lds_probe_kernel(uint32_t iters, uint64_t *out) {
    __shared__ uint64_t s[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += kProbeThreads) s[i] = (uint64_t)i * 0x9e3779b97f4a7c15ull;
    __syncthreads();
    uint64_t a = 0, b = 0;
    uint32_t base = threadIdx.x;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 16; j += 2) {
            a ^= s[base + j * kProbeThreads];
            b += s[base + (j + 1) * kProbeThreads];
        }
        base = (base + 7) & (kProbeThreads - 1);   // keeps lanes on distinct consecutive words
    }
    out[blockIdx.x * kProbeThreads + threadIdx.x] = a ^ b;
}

}  // namespace

hipError_t run_peak_probes(int cu_count, hipStream_t s, double *valu_lane_ops_per_s,
                           double *lds_bytes_per_s) {
    const uint32_t blocks = (uint32_t)cu_count * 8;
    const uint32_t valu_iters = 1u << 14, lds_iters = 1u << 11;
    void *buf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t r = hipMalloc(&buf, (size_t)blocks * kProbeThreads * 8);
    if (r == hipSuccess) r = hipEventCreate(&e0);
    if (r == hipSuccess) r = hipEventCreate(&e1);
    float ms_valu = 0, ms_lds = 0;
    for (int rep = 0; rep < 2 && r == hipSuccess; ++rep) {   // the first pass warms up
        hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, s, 1u, (uint32_t *)buf);
        r = hipEventRecord(e0, s);
        if (r == hipSuccess)
            hipLaunchKernelGGL(valu_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, s, valu_iters,
                               (uint32_t *)buf);
        if (r == hipSuccess) r = hipGetLastError();
        if (r == hipSuccess) r = hipEventRecord(e1, s);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        if (r == hipSuccess) r = hipEventElapsedTime(&ms_valu, e0, e1);
        if (r == hipSuccess) r = hipEventRecord(e0, s);
        if (r == hipSuccess)
            hipLaunchKernelGGL(lds_probe_kernel, dim3(blocks), dim3(kProbeThreads), 0, s, lds_iters,
                               (uint64_t *)buf);
        if (r == hipSuccess) r = hipGetLastError();
        if (r == hipSuccess) r = hipEventRecord(e1, s);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        if (r == hipSuccess) r = hipEventElapsedTime(&ms_lds, e0, e1);
    }
    if (r == hipSuccess) {
        const double lanes = (double)blocks * kProbeThreads;
        *valu_lane_ops_per_s = lanes * valu_iters * kChains / (ms_valu * 1e-3);
        *lds_bytes_per_s = lanes * lds_iters * 16 * 8 / (ms_lds * 1e-3);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (buf) (void)hipFree(buf);
    return r;
}

}  // namespace cuboid
