// Temporal blend over two sets of averages (Section 3.4.1) for gfx950.
// One lane per slot of the current table (grid-stride); lanes whose
// occupancy bit is clear leave at once, so the work beyond a bitmap read is
// proportional to the cells of the current frame.
#include "pf_device.h"
#include "pf_kernels.h"

namespace pfk {

constexpr uint32_t kTemporalGrid = 2048;

// Searches key in a table by fingerprint, confirming with the stored key.
__device__ __forceinline__ uint32_t find_exact(const Tab &t, uint64_t key, uint32_t f) {
    uint32_t s = home_of(key, t.mask);
    for (uint32_t d = 0; d < t.max_probe; ++d) {
        const uint32_t cur = t.cell[s].fp;
        if (cur == 0) return kNoSlot;
        if (cur == f && t.key[s] == key) return s;
        s = (s + 1) & t.mask;
    }
    return kNoSlot;
}

template <bool kHasPrev>
__global__ __launch_bounds__(kBlock) void temporal_kernel(Tab cur, Tab prev, float alpha, float beta) {
    const uint32_t nslots = cur.mask + 1;
    const uint32_t stride = gridDim.x * kBlock;
    uint32_t hits = 0;
    for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < nslots; s += stride) {
        if (((cur.occ[s >> 5] >> (s & 31)) & 1u) == 0) continue;
        const pf_cell c = cur.cell[s];
        float v0 = cell_average(c.sum[0], c.count, cur.frac_bits);
        float v1 = cell_average(c.sum[1], c.count, cur.frac_bits);
        float v2 = cell_average(c.sum[2], c.count, cur.frac_bits);
        if constexpr (kHasPrev) {
            const uint64_t key = cur.key[s];
            const uint32_t p = find_exact(prev, key, c.fp);
            if (p != kNoSlot) {
                const float4 old = prev.blend[p];
                const float a0 = alpha * old.x, a1 = alpha * old.y, a2 = alpha * old.z;
                const float b0 = beta * v0, b1 = beta * v1, b2 = beta * v2;
                v0 = a0 + b0;
                v1 = a1 + b1;
                v2 = a2 + b2;
                ++hits;
            }
        }
        cur.blend[s] = make_float4(v0, v1, v2, (float)c.count);
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
