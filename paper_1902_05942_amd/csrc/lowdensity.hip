// Fallbacks for voxels with few vertices (Section 3.3) for gfx950.
//
// The work is per sparse voxel, not per vertex.  A workgroup takes a range
// of occupancy words and lists in LDS the occupied slots of the range whose
// count is below the threshold; the listed voxels are then searched, each
// writing its pooled average into its temporal value, which the lookup with
// use_blend returns.
//   kMode 0, neighbourhood search: 8 lanes per voxel, lane l searching the
//     keys of candidates 4l .. 4l+3 of the 27 voxels (dx, dy, dz) =
//     (c % 3 - 1, c / 3 % 3 - 1, c / 9 - 1) away at the same level and normal
//     class, its four searches in flight together; the partial sums of the
//     8 lanes are added with cross-lane adds;
//   kMode 1, similar normals along the probe run: one lane per voxel.  The
//     key's home slot does not depend on its normal class, so the voxels at
//     its position and level with other normals lie in its probe run, from
//     the home slot to the first empty one (at most max_probe slots), which
//     the occupancy bitmap shows; the lane reads the keys of that run and
//     counts the voxels with the same position bits whose normal class
//     vector has a positive dot product with its own.
// A key whose home slot is empty is not in the table (linear probing with
// no deletions), and the occupancy bitmap (1 bit per slot, L2-resident) says
// so without a random read of the slot: most candidate neighbours are
// absent.  Sums and counts are pooled as integers (exact, order-free) and
// divided once as the lookup divides: (float)((double)S * 2^-F / (double)N).
#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

constexpr int kLdThreads = 256;
constexpr uint32_t kLdWords = kLdThreads / 4;  // four lanes per occupancy word, 8 slots each
constexpr uint32_t kLdSlots = kLdWords * 32;
constexpr uint32_t kCubeLanes = 8, kCubePer = 4;  // 8 x 4 >= 27 candidates per voxel
constexpr uint64_t kCoordMask = (1ull << 51) - 1;

__device__ __forceinline__ int class_sign(uint64_t key, int axis) {
    const uint32_t v = (uint32_t)(key >> (56 + 2 * axis)) & 3u;
    return v == 1 ? 1 : (v == 2 ? -1 : 0);
}

__device__ __forceinline__ bool occupied(const Tab &t, uint32_t s) { return (t.occ[s >> 5] >> (s & 31)) & 1u; }

__device__ __forceinline__ void add_cell(const Tab &t, uint32_t s, uint32_t &n, uint64_t &a0, uint64_t &a1,
                                         uint64_t &a2) {
    const uint4 *c = t.words_at(s);
    const uint4 lo = c[0], hi = c[1];
    n += lo.y;
    a0 += (uint64_t)lo.z | (uint64_t)lo.w << 32;
    a1 += (uint64_t)hi.x | (uint64_t)hi.y << 32;
    a2 += (uint64_t)hi.z | (uint64_t)hi.w << 32;
}

__device__ __forceinline__ void store_pooled(const Tab &t, uint32_t s, uint32_t n, uint64_t a0, uint64_t a1,
                                             uint64_t a2) {
    float *v = reinterpret_cast<float *>(&t.blend_at(s));
    v[0] = cell_average((int64_t)a0, n, t.frac_bits);
    v[1] = cell_average((int64_t)a1, n, t.frac_bits);
    v[2] = cell_average((int64_t)a2, n, t.frac_bits);
}

// Neighbourhood search for voxel s (key K) by this lane's candidates.
__device__ __forceinline__ void search_cube(const Tab &t, uint32_t s, uint64_t K, uint32_t lane, uint32_t &n,
                                            uint64_t &a0, uint64_t &a1, uint64_t &a2) {
    uint64_t k2[kCubePer];
    uint32_t f[kCubePer], p[kCubePer], found[kCubePer];
    bool act[kCubePer];
#pragma unroll
    for (uint32_t u = 0; u < kCubePer; ++u) {
        const uint32_t c = lane * kCubePer + u;
        const int d[3] = {(int)(c % 3) - 1, (int)(c / 3 % 3) - 1, (int)(c / 9) - 1};
        k2[u] = K & ~kCoordMask;
        bool in = c < 27;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int x = (int)((K >> (17 * a)) & 0x1ffffu) - 65536 + d[a];
            in = in && x > -65536 && x < 65536;
            k2[u] |= (uint64_t)(uint32_t)(x + 65536) << (17 * a);
        }
        found[u] = (in && c == 13) ? s : kNoSlot;  // the voxel itself
        act[u] = in && c != 13;
        p[u] = act[u] ? home_of(k2[u], t.mask) : 0u;
        f[u] = act[u] ? fingerprint_of(k2[u]) : 0u;
    }
#pragma unroll
    for (uint32_t u = 0; u < kCubePer; ++u) act[u] = act[u] && occupied(t, p[u]);
    for (uint32_t d = 0; d < t.max_probe; ++d) {
        bool any = false;
#pragma unroll
        for (uint32_t u = 0; u < kCubePer; ++u) any |= act[u];
        if (!any) break;
        uint32_t cur[kCubePer];
        uint64_t kk[kCubePer];
#pragma unroll
        for (uint32_t u = 0; u < kCubePer; ++u) cur[u] = act[u] ? t.cell_at(p[u]).fp : 0u;
#pragma unroll
        for (uint32_t u = 0; u < kCubePer; ++u) kk[u] = (act[u] && cur[u] == f[u]) ? t.key_at(p[u]) : 0ull;
#pragma unroll
        for (uint32_t u = 0; u < kCubePer; ++u) {
            if (!act[u]) continue;
            if (cur[u] == 0) {
                act[u] = false;
            } else if (cur[u] == f[u] && kk[u] == k2[u]) {
                found[u] = p[u];
                act[u] = false;
            } else {
                p[u] = (p[u] + 1) & t.mask;
            }
        }
    }
#pragma unroll
    for (uint32_t u = 0; u < kCubePer; ++u)
        if (found[u] != kNoSlot) add_cell(t, found[u], n, a0, a1, a2);
}

// Similar normals along the probe run of voxel s (key K), one lane.
__device__ __forceinline__ void search_normals(const Tab &t, uint64_t K, uint32_t &n, uint64_t &a0, uint64_t &a1,
                                               uint64_t &a2) {
    uint32_t p = home_of(K, t.mask);
    for (uint32_t d = 0; d < t.max_probe;) {
        // the occupied slots from p on, up to the next word boundary, in
        // order: the run ends at the first clear bit
        const uint32_t sh = p & 31;
        const uint32_t w = t.occ[p >> 5] >> sh;
        // (a table of fewer than 32 slots wraps inside its only word)
        const uint32_t span = min(min(32 - sh, t.max_probe - d), t.mask + 1 - p);
        const uint32_t run = min(w == 0xffffffffu ? 32u : (uint32_t)__builtin_ctz(~w), span);
        uint64_t kk[4];
        uint32_t done = 0;
        while (done < run) {
            const uint32_t m = min(run - done, 4u);
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) kk[u] = u < m ? t.key_at((p + done + u) & t.mask) : 0ull;
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                if (u >= m) continue;
                int dot = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a) dot += class_sign(K, a) * class_sign(kk[u], a);
                if (((kk[u] ^ K) & kPosMask) == 0 && dot > 0) add_cell(t, (p + done + u) & t.mask, n, a0, a1, a2);
            }
            done += m;
        }
        if (run < span) break;  // an empty slot ends the run
        d += span;
        p = (p + span) & t.mask;
    }
}

template <int kMode>
__global__ __launch_bounds__(kLdThreads) void low_density_kernel(Tab t, uint32_t below) {
    __shared__ uint32_t list[kLdSlots];
    __shared__ uint32_t nlist;
    const uint32_t nwords = t.nwords();
    const uint32_t nranges = (nwords + kLdWords - 1) / kLdWords;
    for (uint32_t rg = blockIdx.x; rg < nranges; rg += gridDim.x) {
        if (threadIdx.x == 0) nlist = 0;
        __syncthreads();
        const uint32_t j = rg * kLdWords + (threadIdx.x >> 2);
        if (j < nwords) {
            // the counts of the lane's (up to 8) occupied slots are loaded together
            const uint32_t b0 = 8 * (threadIdx.x & 3);
            const uint32_t w = (t.occ[j] >> b0) & 0xffu;
            uint32_t cnt[8];
#pragma unroll
            for (uint32_t b = 0; b < 8; ++b) cnt[b] = ((w >> b) & 1u) ? t.cell_at(j * 32 + b0 + b).count : 0u;
#pragma unroll
            for (uint32_t b = 0; b < 8; ++b)
                if (((w >> b) & 1u) && cnt[b] < below) list[atomicAdd(&nlist, 1u)] = j * 32 + b0 + b;
        }
        __syncthreads();
        const uint32_t m = nlist;
        if constexpr (kMode == 0) {
            const uint32_t lane = threadIdx.x % kCubeLanes;
            // the 8 lanes of a voxel share q, so they run the same trips
            // and are all active for the cross-lane sums
            for (uint32_t q = threadIdx.x / kCubeLanes; q < m; q += kLdThreads / kCubeLanes) {
                const uint32_t s = list[q];
                uint32_t n = 0;
                uint64_t a0 = 0, a1 = 0, a2 = 0;
                search_cube(t, s, t.key_at(s), lane, n, a0, a1, a2);
#pragma unroll
                for (uint32_t x = kCubeLanes / 2; x >= 1; x >>= 1) {
                    n += (uint32_t)__shfl_xor((int)n, (int)x);
                    a0 += (uint64_t)__shfl_xor((unsigned long long)a0, (int)x);
                    a1 += (uint64_t)__shfl_xor((unsigned long long)a1, (int)x);
                    a2 += (uint64_t)__shfl_xor((unsigned long long)a2, (int)x);
                }
                if (lane == 0) store_pooled(t, s, n, a0, a1, a2);
            }
        } else {
            for (uint32_t q = threadIdx.x; q < m; q += kLdThreads) {
                const uint32_t s = list[q];
                uint32_t n = 0;
                uint64_t a0 = 0, a1 = 0, a2 = 0;
                search_normals(t, t.key_at(s), n, a0, a1, a2);
                store_pooled(t, s, n, a0, a1, a2);
            }
        }
        __syncthreads();  // the list is rebuilt for the next range
    }
}

hipError_t launch_low_density(const Tab &t, uint32_t below, int mode, hipStream_t st) {
    const uint32_t ranges = (t.nwords() + kLdWords - 1) / kLdWords;
    const uint32_t blocks = ranges < 8192 ? ranges : 8192;
    if (mode == 0)
        low_density_kernel<0><<<blocks, kLdThreads, 0, st>>>(t, below);
    else
        low_density_kernel<1><<<blocks, kLdThreads, 0, st>>>(t, below);
    return hipGetLastError();
}

}  // namespace pfk
