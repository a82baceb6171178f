// A history of voxel values kept beyond the previous frame, with eviction by
// priority (Section 3.4.3), for gfx950.
//
// The history is direct-mapped: the voxel with key K lives only in slot
// fmix64(K) mod 2^h.  A slot is a 32-byte record of a 64-bit word, the key
// and the value (c, N), so a lookup reads one line; the frame it was last
// written lives in a separate array read only when ageing.  The word's top byte is a priority,
// (min(age, 15) << 4) | (15 - min(floor(log2 N), 15)) (recent voxels first,
// then those with more samples), and its low 56 bits SplitMix64(K) mod 2^56;
// an empty slot's word is all ones.  Of the resident and the voxels of a
// frame mapped to a slot, the smallest word stays, so collisions and
// eviction are one 64-bit atomic minimum per voxel and the outcome does not
// depend on the order of arrival.  pf_temporal_history runs four launches:
//   blend    per occupied slot of the frame's table: c_new, the history's
//            (c, N) of its key (one record), the blend of Section 3.4.1,
//            stored in blend;
//   age      per history slot (a dense, coalesced pass): voxels older than
//            max_age are dropped, the others get the word of their age;
//   compete  per occupied slot of the frame's table: atomic minimum of its
//            word (age 0) into its history slot;
//   own      per occupied slot: the voxel whose word is the slot's minimum
//            writes key, value and stamp.
#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

__device__ __forceinline__ uint64_t history_word(uint64_t key, uint32_t age, uint32_t count) {
    const uint32_t a = age < 15 ? age : 15;
    const uint32_t lg = 31 - __builtin_clz(count ? count : 1u);
    const uint32_t p = (a << 4) | (15 - (lg < 15 ? lg : 15));
    return ((uint64_t)p << 56) | (splitmix64(key) & ((1ull << 56) - 1));
}

__device__ __forceinline__ uint32_t history_slot(const Hist &h, uint64_t key) {
    return (uint32_t)(fmix64(key) & h.mask);
}

template <bool kIntegrate>
__global__ __launch_bounds__(kBlock) void history_blend_kernel(Tab cur, Hist h, float alpha, float beta,
                                                               uint32_t cap) {
    const uint32_t nparts = cur.nwords() * 4;
    const uint32_t stride = gridDim.x * kBlock;
    uint32_t hits = 0;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < nparts; q += stride) {
        uint32_t w = cur.occ[q >> 2] & (0xffu << (8 * (q & 3)));
        while (w) {
            const uint32_t s = (q >> 2) * 32 + __builtin_ctz(w);
            w &= w - 1;
            const uint4 *w4 = cur.words_at(s);  // cell and key in one record
            const uint4 lo = w4[0], hi = w4[1], kw = w4[2];
            const uint64_t key = (uint64_t)kw.x | (uint64_t)kw.y << 32;
            pf_cell c;
            c.fp = lo.x;
            c.count = lo.y;
            c.sum[0] = (int64_t)((uint64_t)lo.z | (uint64_t)lo.w << 32);
            c.sum[1] = (int64_t)((uint64_t)hi.x | (uint64_t)hi.y << 32);
            c.sum[2] = (int64_t)((uint64_t)hi.z | (uint64_t)hi.w << 32);
            float v[3] = {cur.average(c, 0), cur.average(c, 1), cur.average(c, 2)};
            uint32_t keep = kIntegrate ? min(c.count, cap) : c.count;
            const uint32_t hs = history_slot(h, key);
            // the slot's word, key and value in one 32-byte record
            const uint4 *rec = reinterpret_cast<const uint4 *>(h.slot + hs);
            const uint4 rw = rec[0], rv = rec[1];
            const uint64_t hw = (uint64_t)rw.x | (uint64_t)rw.y << 32;
            const uint64_t hk = (uint64_t)rw.z | (uint64_t)rw.w << 32;
            const float4 old = make_float4(__uint_as_float(rv.x), __uint_as_float(rv.y), __uint_as_float(rv.z),
                                           __uint_as_float(rv.w));
            if (hw != ~0ull && hk == key) {
                float al = alpha, be = beta;
                if constexpr (kIntegrate) {
                    const float nsum = old.w + (float)c.count;  // exact integers below 2^24
                    al = old.w / nsum;
                    be = 1.0f - al;
                    const uint32_t n = (uint32_t)nsum;
                    keep = n < cap ? n : cap;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float a = al * (k == 0 ? old.x : (k == 1 ? old.y : old.z));
                    const float b = be * v[k];
                    v[k] = a + b;
                }
                ++hits;
            }
            cur.blend_at(s) = make_float4(v[0], v[1], v[2], (float)keep);
        }
    }
    __shared__ uint32_t s_hits;
    if (threadIdx.x == 0) s_hits = 0;
    __syncthreads();
    if (hits) atomicAdd(&s_hits, hits);
    __syncthreads();
    if (threadIdx.x == 0 && s_hits) add_u64(&cur.stats[PF_STAT_PART_HIT + (blockIdx.x & 31)], s_hits);
}

__global__ __launch_bounds__(kBlock) void history_age_kernel(Hist h, uint32_t frame, uint32_t max_age) {
    const uint64_t n = (uint64_t)h.mask + 1;
    for (uint64_t s = (uint64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += (uint64_t)gridDim.x * kBlock) {
        pf_history_slot &r = h.slot[s];
        if (r.word == ~0ull) continue;
        const uint32_t age = frame - h.stamp[s];
        r.word = age > max_age ? ~0ull : history_word(r.key, age, (uint32_t)r.value[3]);
    }
}

// kOwn false: atomic minimum of each voxel's word into its slot; true: the
// voxel holding the slot's minimum writes its key, value and stamp.
template <bool kOwn>
__global__ __launch_bounds__(kBlock) void history_offer_kernel(Tab cur, Hist h, uint32_t frame) {
    const uint32_t nparts = cur.nwords() * 4;
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < nparts; q += stride) {
        uint32_t w = cur.occ[q >> 2] & (0xffu << (8 * (q & 3)));
        while (w) {
            const uint32_t s = (q >> 2) * 32 + __builtin_ctz(w);
            w &= w - 1;
            const uint64_t key = cur.key_at(s);
            const float4 v = cur.blend_at(s);
            const uint64_t mine = history_word(key, 0, (uint32_t)v.w);
            const uint32_t hs = history_slot(h, key);
            if constexpr (!kOwn) {
                atomicMin(reinterpret_cast<unsigned long long *>(&h.slot[hs].word), (unsigned long long)mine);
            } else if (h.slot[hs].word == mine) {
                uint4 *rec = reinterpret_cast<uint4 *>(h.slot + hs);
                rec[0] = make_uint4((uint32_t)mine, (uint32_t)(mine >> 32), (uint32_t)key, (uint32_t)(key >> 32));
                rec[1] = make_uint4(__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z),
                                    __float_as_uint(v.w));
                h.stamp[hs] = frame;
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void history_init_kernel(Hist h) {
    const uint64_t n = (uint64_t)h.mask + 1;
    for (uint64_t s = (uint64_t)blockIdx.x * kBlock + threadIdx.x; s < n; s += (uint64_t)gridDim.x * kBlock)
        h.slot[s].word = ~0ull;  // empty; key, value and stamp are written with the word that owns them
}

hipError_t launch_history_init(const Hist &h, hipStream_t st) {
    const uint64_t n = (uint64_t)h.mask + 1;
    uint64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    history_init_kernel<<<(uint32_t)blocks, kBlock, 0, st>>>(h);
    return hipGetLastError();
}

hipError_t launch_temporal_history(const Tab &cur, const Hist &h, float alpha_old, int mode, uint32_t cap,
                                   uint32_t frame, hipStream_t st) {
    const uint32_t parts = cur.nwords() * 4;
    uint32_t blocks = (parts + kBlock - 1) / kBlock;
    if (blocks > 16384) blocks = 16384;
    if (mode == 1)
        history_blend_kernel<true><<<blocks, kBlock, 0, st>>>(cur, h, 0.0f, 0.0f, cap);
    else
        history_blend_kernel<false><<<blocks, kBlock, 0, st>>>(cur, h, alpha_old, 1.0f - alpha_old, cap);
    const uint64_t n = (uint64_t)h.mask + 1;
    uint64_t ablocks = (n + kBlock - 1) / kBlock;
    if (ablocks > 8192) ablocks = 8192;
    history_age_kernel<<<(uint32_t)ablocks, kBlock, 0, st>>>(h, frame, h.max_age);
    history_offer_kernel<false><<<blocks, kBlock, 0, st>>>(cur, h, frame);
    history_offer_kernel<true><<<blocks, kBlock, 0, st>>>(cur, h, frame);
    return hipGetLastError();
}

}  // namespace pfk
