// Temporal blend over two sets of averages (Section 3.4.1) for gfx950: four
// lanes per occupancy word of the current table (temporal_word), so the work
// beyond the bitmap read is proportional to the cells of the current frame.
#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

template <bool kHasPrev, bool kIntegrate, bool kLevels = false>
__global__ __launch_bounds__(kBlock) void temporal_kernel(Tab cur, Tab prev, float alpha, float beta, uint32_t cap) {
    // four lanes per occupancy word, 8 slots each: enough lanes in flight to
    // hide the chain of dependent lookups
    const uint32_t nparts = cur.nwords() * 4;
    const uint32_t stride = gridDim.x * kBlock;
    uint32_t hits = 0;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < nparts; q += stride)
        hits += temporal_word<kHasPrev, kIntegrate, 2, kLevels>(cur, prev, q >> 2, alpha, beta, cap,
                                                                 0xffu << (8 * (q & 3)));
    if constexpr (kHasPrev) {
        // one device atomic per block, spread over 32 partial counters
        __shared__ uint32_t s_hits;
        if (threadIdx.x == 0) s_hits = 0;
        __syncthreads();
        if (hits) atomicAdd(&s_hits, hits);
        __syncthreads();
        if (threadIdx.x == 0 && s_hits) add_u64(&cur.stats[PF_STAT_PART_HIT + (blockIdx.x & 31)], s_hits);
    }
}

hipError_t launch_temporal(const Tab &cur, const Tab *prev, float alpha_old, int mode, uint32_t cap,
                           hipStream_t st) {
    const float beta = 1.0f - alpha_old;
    uint32_t blocks = (cur.nwords() * 4 + kBlock - 1) / kBlock;
    if (blocks > 16384) blocks = 16384;
    const bool levels = (mode & PF_TEMPORAL_ACROSS_LEVELS) != 0;
    mode &= ~PF_TEMPORAL_ACROSS_LEVELS;
    if (levels && prev) {  // without a previous table there is nothing to search
        if (mode == 1)
            temporal_kernel<true, true, true><<<blocks, kBlock, 0, st>>>(cur, *prev, 0.0f, 0.0f, cap);
        else
            temporal_kernel<true, false, true><<<blocks, kBlock, 0, st>>>(cur, *prev, alpha_old, beta, cap);
    } else if (mode == 1) {
        if (prev)
            temporal_kernel<true, true><<<blocks, kBlock, 0, st>>>(cur, *prev, 0.0f, 0.0f, cap);
        else
            temporal_kernel<false, true><<<blocks, kBlock, 0, st>>>(cur, cur, 0.0f, 0.0f, cap);
    } else {
        if (prev)
            temporal_kernel<true, false><<<blocks, kBlock, 0, st>>>(cur, *prev, alpha_old, beta, cap);
        else
            temporal_kernel<false, false><<<blocks, kBlock, 0, st>>>(cur, cur, alpha_old, beta, cap);
    }
    return hipGetLastError();
}

}  // namespace pfk
