// Microbenchmark of LDS atomic throughput on the device (the vote's LDS ceiling).
//
// One 1,024-thread workgroup per CU with the sweep's 160 KB LDS allocation; every
// lane issues ds_add_u32 of 1 in a loop, either to 64 distinct banks (lane i ->
// word thread + 1,024 r + 8,192 (it mod 4): conflict-free) or to pseudo-random
// words (a per-lane draw XOR a per-iteration value), the access pattern of the
// vote.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "host.h"

namespace dses {
namespace {

constexpr int kProbeWords = 40960;

template <int PATTERN>
__global__ void __launch_bounds__(1024) k_lds_add(int32_t iters, uint32_t *sink)
{
    __shared__ uint32_t lds[kProbeWords];
    const int tid = threadIdx.x;
    for (int w = tid; w < kProbeWords; w += 1024) lds[w] = 0u;
    __syncthreads();
    // addresses stay in the first 32,768 words; at most 2 VALU per add, so the
    // loop is bound by the LDS, not by the address arithmetic
    uint32_t word[8];
    uint32_t x = 2654435761u * (uint32_t)(tid + 1) + 97u * blockIdx.x;
    const uint32_t base = (uint32_t)(size_t)(__attribute__((address_space(3))) uint32_t *)lds;
#pragma unroll
    for (int r = 0; r < 8; ++r) {           // byte offsets below 128 KB
        x = x * 1664525u + 1013904223u;
        word[r] = 4u * (PATTERN == 0 ? (uint32_t)tid + 1024u * (uint32_t)r : (x >> 9) & 32767u);
    }
    for (int it = 0; it < iters; ++it) {
        // the same change for every lane of the workgroup: another bank-free layout
        // (pattern 0: the word offset gains a multiple of 8,192, keeping each lane's
        // bank) or another random permutation (pattern 1); one VALU per add
        const uint32_t s = PATTERN == 0 ? 32768u * (uint32_t)(it & 3)
                                        : (((uint32_t)it * 2654435761u) & 32767u) << 2;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint32_t addr = base + (word[r] ^ s);
            asm volatile("ds_add_u32 %0, %1" ::"v"(addr), "v"(1u) : "memory");
        }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __syncthreads();
    if (tid == 0) sink[blockIdx.x] = lds[blockIdx.x % kProbeWords];
}

}  // namespace
}  // namespace dses

using namespace dses;

extern "C" dses_status dses_measure_lds_atomics(int32_t pattern, double *adds_per_second,
                                                double *per_cu_per_cycle)
{
    set_error("");
    if ((pattern != 0 && pattern != 1) || !adds_per_second) {
        set_error("pattern must be 0 (conflict-free) or 1 (random) with an output pointer");
        return DSES_E_INVAL;
    }
    Context *c = ctx();
    if (!c) return DSES_E_DEVICE;
    std::lock_guard<std::mutex> lk(c->mu);
    const int grid = c->n_cu;
    const int32_t iters = 4096;                       // 8 adds per iteration per lane
    uint32_t *sink = nullptr;
    DSES_HIP(dev_alloc(&sink, grid * sizeof(uint32_t)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DSES_HIP(hipEventCreate(&e0));
    DSES_HIP(hipEventCreate(&e1));
    auto launch = [&]() {
        if (pattern == 0)
            hipLaunchKernelGGL(k_lds_add<0>, dim3(grid), dim3(1024), 0, c->stream, iters, sink);
        else
            hipLaunchKernelGGL(k_lds_add<1>, dim3(grid), dim3(1024), 0, c->stream, iters, sink);
    };
    launch();                                          // warm-up
    DSES_HIP(hipEventRecord(e0, c->stream));
    launch();
    DSES_HIP(hipEventRecord(e1, c->stream));
    DSES_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    DSES_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    const double adds = (double)grid * 1024.0 * iters * 8.0;
    *adds_per_second = adds / (ms * 1e-3);
    if (per_cu_per_cycle) {
        int khz = 0;
        (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, c->device);
        *per_cu_per_cycle = khz > 0 ? *adds_per_second / grid / (khz * 1e3) : 0.0;
    }
    return DSES_OK;
}
