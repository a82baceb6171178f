// Temporal blend over two sets of averages (Section 3.4.1) for gfx950.
// One lane per slot of the current table (grid-stride); lanes whose
// occupancy bit is clear leave at once, so the work beyond a bitmap read is
// proportional to the cells of the current frame.
#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

constexpr uint32_t kTemporalGrid = 2048;

template <bool kHasPrev>
__global__ __launch_bounds__(kBlock) void temporal_kernel(Tab cur, Tab prev, float alpha, float beta) {
    const uint32_t nslots = cur.mask + 1;
    const uint32_t stride = gridDim.x * kBlock;
    uint32_t hits = 0;
    for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < nslots; s += stride) {
        if (((cur.occ[s >> 5] >> (s & 31)) & 1u) == 0) continue;
        hits += temporal_cell<kHasPrev>(cur, prev, s, alpha, beta) ? 1u : 0u;
    }
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

hipError_t launch_temporal(const Tab &cur, const Tab *prev, float alpha_old, int mode, hipStream_t st) {
    (void)mode;
    const float beta = 1.0f - alpha_old;
    if (prev)
        temporal_kernel<true><<<kTemporalGrid, kBlock, 0, st>>>(cur, *prev, alpha_old, beta);
    else
        temporal_kernel<false><<<kTemporalGrid, kBlock, 0, st>>>(cur, cur, alpha_old, beta);
    return hipGetLastError();
}

}  // namespace pfk
