// Temporal blend over two sets of averages (Section 3.4.1) for gfx950.
// One lane per occupancy word of the current table: its occupied slots are
// taken four at a time, and each step of their lookups in the previous
// table (cell and key, fingerprint probe, key check, old value) is issued
// for all four before any result is used, so a lane waits for four
// dependent round trips per four cells instead of per cell.  Work beyond
// the bitmap read is proportional to the cells of the current frame.
#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

constexpr int kTB = 4;  // cells of one lane looked up together

// kIntegrate: temporal integration, alpha = N_old / (N_old + N_new) per cell
// with the stored count kept at most `cap`; else the moving average with a
// fixed alpha (the stored count is this frame's).
template <bool kHasPrev, bool kIntegrate>
__global__ __launch_bounds__(kBlock) void temporal_kernel(Tab cur, Tab prev, float alpha, float beta, uint32_t cap) {
    const uint32_t nwords = cur.nwords();
    const uint32_t stride = gridDim.x * kBlock;
    const uint4 *cells = reinterpret_cast<const uint4 *>(cur.cell);
    uint32_t hits = 0;
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < nwords; j += stride) {
        uint32_t w = cur.occ[j];
        while (w) {
            uint32_t s[kTB];
            bool has[kTB];
#pragma unroll
            for (int k = 0; k < kTB; ++k) {
                has[k] = w != 0;
                s[k] = has[k] ? j * 32 + __builtin_ctz(w) : 0u;
                w &= w - 1;
            }
            uint4 lo[kTB], hi[kTB];
            uint64_t key[kTB];
#pragma unroll
            for (int k = 0; k < kTB; ++k) {
                if (has[k]) {
                    lo[k] = cells[2 * s[k]];
                    hi[k] = cells[2 * s[k] + 1];
                    if constexpr (kHasPrev) key[k] = cur.key[s[k]];
                }
            }
            float v[kTB][3];
            uint32_t cnt[kTB], keep[kTB];
#pragma unroll
            for (int k = 0; k < kTB; ++k) {
                if (!has[k]) continue;
                pf_cell c;
                c.fp = lo[k].x;
                c.count = lo[k].y;
                c.sum[0] = (int64_t)((uint64_t)lo[k].z | (uint64_t)lo[k].w << 32);
                c.sum[1] = (int64_t)((uint64_t)hi[k].x | (uint64_t)hi[k].y << 32);
                c.sum[2] = (int64_t)((uint64_t)hi[k].z | (uint64_t)hi[k].w << 32);
                cnt[k] = c.count;
                keep[k] = kIntegrate ? min(c.count, cap) : c.count;
                v[k][0] = cur.average(c, 0);
                v[k][1] = cur.average(c, 1);
                v[k][2] = cur.average(c, 2);
            }
            if constexpr (kHasPrev) {
                // search each key in prev: fingerprint probe confirmed by the stored key
                uint32_t p[kTB];
                bool active[kTB], found[kTB];
#pragma unroll
                for (int k = 0; k < kTB; ++k) {
                    active[k] = has[k];
                    found[k] = false;
                    p[k] = has[k] ? home_of(key[k], prev.mask) : 0u;
                }
                for (uint32_t d = 0; d < prev.max_probe; ++d) {
                    bool any = false;
#pragma unroll
                    for (int k = 0; k < kTB; ++k) any |= active[k];
                    if (!any) break;
                    uint32_t pf[kTB];
                    uint64_t pk[kTB];
#pragma unroll
                    for (int k = 0; k < kTB; ++k) pf[k] = active[k] ? prev.cell[p[k]].fp : 0u;
#pragma unroll
                    for (int k = 0; k < kTB; ++k) {
                        pk[k] = 0;
                        if (active[k] && pf[k] == lo[k].x) pk[k] = prev.key[p[k]];
                    }
#pragma unroll
                    for (int k = 0; k < kTB; ++k) {
                        if (!active[k]) continue;
                        if (pf[k] == 0) {
                            active[k] = false;  // empty slot: not in prev
                        } else if (pf[k] == lo[k].x && pk[k] == key[k]) {
                            active[k] = false;
                            found[k] = true;
                        } else {
                            p[k] = (p[k] + 1) & prev.mask;
                        }
                    }
                }
                float4 old[kTB];
#pragma unroll
                for (int k = 0; k < kTB; ++k)
                    if (found[k]) old[k] = prev.blend[p[k]];
#pragma unroll
                for (int k = 0; k < kTB; ++k) {
                    if (!found[k]) continue;
                    float al = alpha, be = beta;
                    if constexpr (kIntegrate) {
                        // counts are exact integers in binary32 (at most 2^24)
                        const float nsum = old[k].w + (float)cnt[k];
                        al = old[k].w / nsum;
                        be = 1.0f - al;
                        const uint32_t n = (uint32_t)nsum;
                        keep[k] = n < cap ? n : cap;
                    }
                    const float a0 = al * old[k].x, a1 = al * old[k].y, a2 = al * old[k].z;
                    const float b0 = be * v[k][0], b1 = be * v[k][1], b2 = be * v[k][2];
                    v[k][0] = a0 + b0;
                    v[k][1] = a1 + b1;
                    v[k][2] = a2 + b2;
                    ++hits;
                }
            }
#pragma unroll
            for (int k = 0; k < kTB; ++k)
                if (has[k]) cur.blend[s[k]] = make_float4(v[k][0], v[k][1], v[k][2], (float)keep[k]);
        }
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

hipError_t launch_temporal(const Tab &cur, const Tab *prev, float alpha_old, int mode, uint32_t cap,
                           hipStream_t st) {
    const float beta = 1.0f - alpha_old;
    uint32_t blocks = (cur.nwords() + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    if (mode == 1) {
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
