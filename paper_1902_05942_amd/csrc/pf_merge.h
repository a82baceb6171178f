// Merging of vertices that share a key inside a workgroup before they touch
// the table, shared by the binned insert (binned.hip) and the batched
// multi-view launch (views.hip): vertices merge by key in an LDS hash table
// of (key, count, fixed-point sums) entries, optionally after runs of equal
// keys across a wavefront's lanes are summed with DPP.
#pragma once

#include "pf_device.h"

namespace pfk {

constexpr uint64_t kEmpty = ~0ull;  // no key has bit 63 set
constexpr uint32_t kLdsProbe = 32;  // LDS probes before a vertex goes alone

// Index of this lane among the lanes of its wavefront that pass want=true,
// the lowest of them reserving the whole range on *ctr.  Every lane of the
// wavefront must call.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t *ctr, bool want) {
    const uint64_t m = __ballot(want);
    const uint32_t rank =
        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    uint32_t base = 0;
    if (m != 0) {
        const int leader = __builtin_ctzll(m);
        if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m));
        base = __shfl(base, leader);
    }
    return base + rank;
}

// LDS entry of `key` in the chunk's table (inserted if absent), or -1 when
// kLdsProbe entries in a row hold other keys.
__device__ __forceinline__ int lds_insert(unsigned long long *lkey, uint32_t cap, uint64_t key) {
    uint32_t j = (uint32_t)(((uint64_t)(uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 32) * cap) >> 32);
#pragma unroll 1
    for (uint32_t d = 0; d < kLdsProbe; ++d) {
        const unsigned long long old = atomicCAS(&lkey[j], (unsigned long long)kEmpty, (unsigned long long)key);
        if (old == kEmpty || old == key) return (int)j;
        j = j + 1 == cap ? 0 : j + 1;
    }
    return -1;
}

// Value of another lane through the DPP crossbar (a VALU operation, no LDS
// round trip): lanes whose source is outside the pattern, or whose row is
// masked off, read 0.
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xf, kRowMask == 0xf);
}
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ uint64_t dpp(uint64_t v) {
    return (uint64_t)dpp<kCtrl, kRowMask>((uint32_t)v) | (uint64_t)dpp<kCtrl, kRowMask>((uint32_t)(v >> 32)) << 32;
}
// a += the DPP source lane's a, as two 32-bit adds chained by the carry
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ void dpp_add(uint64_t &a) {
    const uint32_t lo = (uint32_t)a, hi = (uint32_t)(a >> 32);
    const uint32_t nlo = lo + dpp<kCtrl, kRowMask>(lo);
    const uint32_t nhi = hi + dpp<kCtrl, kRowMask>(hi) + (nlo < lo ? 1u : 0u);
    a = (uint64_t)nlo | (uint64_t)nhi << 32;
}
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ void dpp_add(uint64_t &a0, uint64_t &a1, uint64_t &a2) {
    dpp_add<kCtrl, kRowMask>(a0);
    dpp_add<kCtrl, kRowMask>(a1);
    dpp_add<kCtrl, kRowMask>(a2);
}

// Adds one vertex per lane (lanes with ok) to the chunk's LDS table and
// returns its entry (-1: no room).  kWaveRuns: the lanes of a wavefront hold
// consecutive vertices, so runs of lanes with equal keys (coherent primary
// hits) are summed across the wavefront first and only the last lane of a
// run touches the LDS table: a run's total is the wavefront's inclusive
// prefix sum at its last lane minus the exclusive prefix sum at its first
// (integer sums, exact modulo 2^64); every lane of the wavefront must call.
// Otherwise every valid lane adds itself with LDS atomics.
template <bool kWaveRuns = true>
__device__ __forceinline__ int merge_into_lds(unsigned long long *lkey, unsigned long long *ls0,
                                              unsigned long long *ls1, unsigned long long *ls2, uint32_t *lcnt,
                                              uint32_t cap, bool ok, uint64_t k, int64_t q0, int64_t q1,
                                              int64_t q2) {
    if constexpr (!kWaveRuns) {  // every valid lane adds itself
        int e = -1;
        if (ok) {
            e = lds_insert(lkey, cap, k);
            if (e >= 0) {
                atomicAdd(&lcnt[e], 1u);
                atomicAdd(&ls0[e], (unsigned long long)q0);
                atomicAdd(&ls1[e], (unsigned long long)q1);
                atomicAdd(&ls2[e], (unsigned long long)q2);
            }
        }
        return e;
    }
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t kv = ok ? k : kEmpty;
    const uint64_t prev = dpp<0x138>(kv);  // wave_shr:1, the previous lane's key
    const bool head = lane == 0 || prev != kv;
    const uint64_t heads = __ballot(head);
    const uint64_t upto = (2ull << lane) - 1;  // lanes 0 .. lane
    const uint64_t later = heads & ~upto;
    const uint32_t tail = later ? (uint32_t)__builtin_ctzll(later) - 1 : 63u;  // last lane of my run
    uint32_t cnt = ok ? 1u : 0u;
    uint64_t a0 = (uint64_t)q0, a1 = (uint64_t)q1, a2 = (uint64_t)q2;
    if (__ballot(ok && !head)) {  // some run spans several lanes
        const uint32_t first = 63u - (uint32_t)__builtin_clzll(heads & upto);
        uint64_t p0 = a0, p1 = a1, p2 = a2;
        dpp_add<0x111>(p0, p1, p2);  // row_shr:1
        dpp_add<0x112>(p0, p1, p2);  // row_shr:2
        dpp_add<0x114>(p0, p1, p2);  // row_shr:4
        dpp_add<0x118>(p0, p1, p2);  // row_shr:8
        dpp_add<0x142, 0xa>(p0, p1, p2);  // row_bcast:15 into rows 1 and 3
        dpp_add<0x143, 0xc>(p0, p1, p2);  // row_bcast:31 into rows 2 and 3
        // exclusive prefix at the run's first lane; a run of valid lanes
        // holds only valid lanes (invalid ones carry kEmpty)
        const uint64_t e0 = __shfl((unsigned long long)(p0 - a0), (int)first);
        const uint64_t e1 = __shfl((unsigned long long)(p1 - a1), (int)first);
        const uint64_t e2 = __shfl((unsigned long long)(p2 - a2), (int)first);
        cnt = ok ? tail - first + 1 : 0u;
        a0 = p0 - e0;
        a1 = p1 - e1;
        a2 = p2 - e2;
    }
    int e = -1;
    if (ok && lane == tail) {
        e = lds_insert(lkey, cap, kv);
        if (e >= 0) {
            atomicAdd(&lcnt[e], cnt);
            atomicAdd(&ls0[e], (unsigned long long)a0);
            atomicAdd(&ls1[e], (unsigned long long)a1);
            atomicAdd(&ls2[e], (unsigned long long)a2);
        }
    }
    e = __shfl(e, (int)tail);
    return ok ? e : -1;
}

}  // namespace pfk
