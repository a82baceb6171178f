// Grid-wide barrier for cooperative launches of resident workgroups on
// gfx950 (used by the multi-view launch and the multi-step training launch).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {
namespace grid {

constexpr int kSubCounters = 64;     // first level of the grid barrier
constexpr int kCounterStride = 16;   // uint32 words between counters (64 B)

struct Barrier {
    uint32_t *status;   // [0] non-zero once a wait has timed out
    uint32_t *sub;      // kSubCounters arrival counters, kCounterStride apart
    uint32_t *rel;      // kSubCounters release flags, kCounterStride apart
    uint32_t *top;      // sub-groups arrived
    uint64_t limit;     // wall-clock ticks a wait may last
};

// Reads a counter at the coherence point with a read-modify-write that adds
// 0: loads may be served by an XCD's L2, which does not see atomics made
// elsewhere.  The zero is hidden from the optimiser, which would otherwise
// turn the idempotent read-modify-write back into a plain load.
__device__ __forceinline__ uint32_t poll(uint32_t *p) {
    uint32_t zero = 0;
    asm volatile("" : "+v"(zero));
    return __hip_atomic_fetch_add(p, zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier number `epoch` (1, 2, 3 ...).  A workgroup arrives at
// one of 64 sub-counters; the last arrival of a sub-group advances the top
// counter, waits for all sub-groups, then raises its sub-group's release
// flag, on which the other members wait.  So at most ~64 workgroups poll any
// one address.  Release/acquire fences make the phase's writes visible
// across XCDs.  Every wait is bounded in wall-clock time; a timed-out wait
// sets the status word and returns false (the workgroup then leaves).
__device__ inline bool grid_barrier(const Barrier &bar, uint32_t epoch) {
    __shared__ uint32_t s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t G = gridDim.x;
        const uint32_t nsub = G < (uint32_t)kSubCounters ? G : (uint32_t)kSubCounters;
        const uint32_t sub = blockIdx.x % nsub;
        const uint32_t in_sub = (G - sub + nsub - 1) / nsub;  // workgroups of this sub-group
        const uint32_t old = __hip_atomic_fetch_add(bar.sub + sub * kCounterStride, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        uint32_t ok = 1;
        if (old + 1 == epoch * in_sub) {
            __hip_atomic_fetch_add(bar.top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while (poll(bar.top) < epoch * nsub) {
                if (wall_clock64() - t0 > bar.limit) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
            __hip_atomic_fetch_max(bar.rel + sub * kCounterStride, ok ? epoch : 0xffffffffu, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            for (;;) {
                const uint32_t r = poll(bar.rel + sub * kCounterStride);
                if (r == 0xffffffffu) {
                    ok = 0;
                    break;
                }
                if (r >= epoch) break;
                if (wall_clock64() - t0 > bar.limit) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        if (!ok) {
            __hip_atomic_fetch_or(bar.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(bar.status + 2, poll(bar.top), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(bar.status + 3, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Words of barrier state (status, sub-counters, release flags, top counter),
// zeroed before each launch; the counters are kCounterStride words apart.
constexpr uint32_t kWords = kCounterStride * (2 + 2 * kSubCounters);

__host__ __device__ inline Barrier barrier_at(uint32_t *ws, uint64_t limit) {
    Barrier bar;
    bar.status = ws;
    bar.sub = ws + kCounterStride;
    bar.rel = ws + kCounterStride * (1 + kSubCounters);
    bar.top = ws + kCounterStride * (1 + 2 * kSubCounters);
    bar.limit = limit;
    return bar;
}

}  // namespace grid
}  // namespace pfk
