// Per-vertex and per-cell operations of the filter, shared by the single-view
// kernels (keys.hip, table.hip, temporal.hip) and the batched multi-view
// kernel (views.hip), so every launch shape runs the same arithmetic.
#pragma once

#include "pf_device.h"

#pragma clang fp contract(off)

namespace pfk {

// Key construction of Algorithm 1 for one vertex.  Returns the vertex flags
// (0, PF_V_INVALID or PF_V_KEYRANGE); key/fp/home are 0 for flagged vertices.
// jp holds the launch's PCG32 streams (seed, idx_base) and i is the vertex's
// index within the launch (stream idx_base + i); inv_s = RN(1 / s).
__device__ __forceinline__ uint8_t vertex_key(const float x[3], const float nr[3], bool valid, const float cam[3],
                                              float s, float inv_s, const PcgJump &jp, uint32_t i, uint32_t mask,
                                              uint64_t &key, uint32_t &fp, uint32_t &home) {
    key = 0;
    fp = 0;
    home = 0;
    const bool ok_in = valid && isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(nr[0]) &&
                       isfinite(nr[1]) && isfinite(nr[2]);
    if (!ok_in) return PF_V_INVALID;
    // l <- level_of_detail(|p_cam - x|)
    const int l = level_of_detail(cam[0], cam[1], cam[2], x[0], x[1], x[2]);
    // jitter(n): cube sample projected onto the tangent plane
    float r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = ldexpf((float)(jp.output(c, i) >> 8), -24) - 0.5f;
    const float t0 = r[0] * nr[0];
    const float t1 = r[1] * nr[1];
    const float t2 = r[2] * nr[2];
    const float t = (t0 + t1) + t2;
    // x' <- x + jitter(n) * s * 2^l
    const float h = ldexpf(s, l);
    float xp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float tn = t * nr[c];
        const float j = r[c] - tn;
        const float jh = j * h;
        xp[c] = x[c] + jh;
    }
    // l' <- level_of_detail(|p_cam - x'|); x~ <- floor(x' / (s * 2^l'))
    const int lp = level_of_detail(cam[0], cam[1], cam[2], xp[0], xp[1], xp[2]);
    const float hp = ldexpf(s, lp);
    const float rp = ldexpf(inv_s, -lp);
    bool inrange = true;
    int32_t q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float f = floor_quotient(xp[c], hp, rp);
        inrange = inrange && (f > -kCellIndexLimit) && (f < kCellIndexLimit);  // |x~| < 2^16
        q[c] = inrange ? (int32_t)f : 0;
    }
    if (!inrange) return PF_V_KEYRANGE;
    const uint32_t code = normal_class(nr[0]) | (normal_class(nr[1]) << 2) | (normal_class(nr[2]) << 4);
    key = (uint64_t)(uint32_t)(q[0] + 65536) | ((uint64_t)(uint32_t)(q[1] + 65536) << 17) |
          ((uint64_t)(uint32_t)(q[2] + 65536) << 34) | ((uint64_t)(uint32_t)(lp + 16) << 51) | ((uint64_t)code << 56);
    home = home_of(key, mask);
    fp = fingerprint_of(key);
    return 0;
}

// Fixed-point contribution q_c = rint(c * 2^F).  Returns 0, PF_V_INVALID
// (non-finite) or PF_V_RADRANGE (|c 2^F| >= 2^62).
__device__ __forceinline__ uint8_t fixed_point(float c0, float c1, float c2, int frac_bits, int64_t &q0, int64_t &q1,
                                               int64_t &q2) {
    q0 = q1 = q2 = 0;
    if (!(isfinite(c0) && isfinite(c1) && isfinite(c2))) return PF_V_INVALID;
    const float s0 = ldexpf(c0, frac_bits), s1 = ldexpf(c1, frac_bits), s2 = ldexpf(c2, frac_bits);
    const float lim = 4611686018427387904.0f;  // 2^62
    if (!(fabsf(s0) < lim && fabsf(s1) < lim && fabsf(s2) < lim)) return PF_V_RADRANGE;
    // the active lanes convert through int32 when all of them can (the
    // usual magnitudes): the same integers, a quarter of the instructions
    const float r0 = rintf(s0), r1 = rintf(s1), r2 = rintf(s2);
    const float lim32 = 2147483648.0f;  // 2^31
    if (__builtin_expect(__ballot(!(fabsf(r0) < lim32 && fabsf(r1) < lim32 && fabsf(r2) < lim32)) == 0, 1)) {
        q0 = (int32_t)r0;
        q1 = (int32_t)r1;
        q2 = (int32_t)r2;
    } else {
        q0 = (int64_t)r0;
        q1 = (int64_t)r1;
        q2 = (int64_t)r2;
    }
    return 0;
}

// Contribution kept as binary32 (PF_SUMS_FLOAT32): 0 or PF_V_INVALID.
__device__ __forceinline__ uint8_t float_contribution(float c0, float c1, float c2, float &v0, float &v1, float &v2) {
    v0 = v1 = v2 = 0.0f;
    if (!(isfinite(c0) && isfinite(c1) && isfinite(c2))) return PF_V_INVALID;
    v0 = c0;
    v1 = c1;
    v2 = c2;
    return 0;
}

// One binary32 atomic add per component (the hardware's global_atomic_add_f32).
__device__ __forceinline__ void accumulate(const Tab &t, uint32_t slot, uint32_t cnt, float v0, float v1, float v2) {
    pf_cell *c = &t.cell_at(slot);
    add_u32(&c->count, cnt);
    unsafeAtomicAdd(float_sum(c, 0), v0);
    unsafeAtomicAdd(float_sum(c, 1), v1);
    unsafeAtomicAdd(float_sum(c, 2), v2);
}

__device__ __forceinline__ void accumulate(const Tab &t, uint32_t slot, uint32_t cnt, int64_t q0, int64_t q1,
                                           int64_t q2) {
    pf_cell *c = &t.cell_at(slot);
    add_u32(&c->count, cnt);
    add_u64(reinterpret_cast<unsigned long long *>(&c->sum[0]), (unsigned long long)q0);
    add_u64(reinterpret_cast<unsigned long long *>(&c->sum[1]), (unsigned long long)q1);
    add_u64(reinterpret_cast<unsigned long long *>(&c->sum[2]), (unsigned long long)q2);
}

// Probes from home(key) for the key's fingerprint or claims the first empty
// cell.  Returns the slot or kNoSlot after max_probe slots.  A stale read of
// 0 only leads to a compare-and-swap that returns the current value; a
// non-zero fingerprint never changes within a kernel.
__device__ __forceinline__ uint32_t find_or_claim(const Tab &t, uint64_t key) {
    const uint32_t f = fingerprint_of(key);
    uint32_t s = home_of(key, t.mask);
    for (uint32_t d = 0; d < t.max_probe; ++d) {
        uint32_t *pfp = &t.cell_at(s).fp;
        uint32_t cur = load_fp_probe(pfp);
        if (cur == 0) {
            uint32_t expected = 0;
            if (__hip_atomic_compare_exchange_strong(pfp, &expected, f, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                t.key_at(s) = key;
                __hip_atomic_fetch_or(&t.occ[s >> 5], 1u << (s & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return s;
            }
            cur = expected;  // claimed meanwhile by someone else
        }
        if (cur == f) return s;
        s = (s + 1) & t.mask;
    }
    return kNoSlot;
}

// Probe without claiming (lookup after insertion).
__device__ __forceinline__ uint32_t find_slot(const Tab &t, uint64_t key) {
    const uint32_t f = fingerprint_of(key);
    uint32_t s = home_of(key, t.mask);
    for (uint32_t d = 0; d < t.max_probe; ++d) {
        const uint32_t cur = t.cell_at(s).fp;
        if (cur == f) return s;
        if (cur == 0) return kNoSlot;
        s = (s + 1) & t.mask;
    }
    return kNoSlot;
}

// Search by fingerprint confirmed with the stored 64-bit key.
__device__ __forceinline__ uint32_t find_exact(const Tab &t, uint64_t key, uint32_t f) {
    uint32_t s = home_of(key, t.mask);
    for (uint32_t d = 0; d < t.max_probe; ++d) {
        const uint32_t cur = t.cell_at(s).fp;
        if (cur == 0) return kNoSlot;
        if (cur == f && t.key_at(s) == key) return s;
        s = (s + 1) & t.mask;
    }
    return kNoSlot;
}

// LDS scratch of the workgroup aggregation (kBlockT threads).
template <int kBlockT>
struct AggLds {
    uint32_t bucket[2 * kBlockT];
    uint32_t slot[kBlockT];
    unsigned long long acc[3][kBlockT];
    uint32_t cnt[kBlockT];
};

// Accumulates every lane's contribution into its slot.  agg <= 1: one set of
// device atomics per lane.  agg > 1 (power of two <= kBlockT): lanes of an
// aggregation group (agg consecutive threads) that reach the same slot first
// add their contributions in LDS; one lane per (group, slot) then issues the
// device atomics.  Groups meet through a bucket array indexed by the slot's
// low bits; a lane whose bucket was taken by another slot goes direct.  Must
// be reached by every thread of the workgroup when agg > 1.
__device__ __forceinline__ void lds_add(unsigned long long *p, int64_t v) { atomicAdd(p, (unsigned long long)v); }
__device__ __forceinline__ void lds_add(unsigned long long *p, float v) { atomicAdd(reinterpret_cast<float *>(p), v); }
__device__ __forceinline__ int64_t lds_value(const unsigned long long *p, int64_t) { return (int64_t)*p; }
__device__ __forceinline__ float lds_value(const unsigned long long *p, float) {
    return *reinterpret_cast<const float *>(p);
}

// V is int64_t (fixed-point sums) or float (binary32 sums, in the low word
// of each LDS accumulator).
template <int kBlockT, typename V>
__device__ __forceinline__ void accumulate_group(const Tab &t, AggLds<kBlockT> &L, uint32_t agg, uint32_t slot,
                                                 V q0, V q1, V q2) {
    const bool has = slot != kNoSlot;
    if (agg <= 1) {
        if (has) accumulate(t, slot, 1, q0, q1, q2);
        return;
    }
    const uint32_t tid = threadIdx.x;
    const uint32_t gbase = tid & ~(agg - 1);  // first lane of my group
    L.slot[tid] = slot;
    L.acc[0][tid] = 0;
    L.acc[1][tid] = 0;
    L.acc[2][tid] = 0;
    L.cnt[tid] = 0;
    // every lane with a slot writes its id into its bucket; one write wins
    const uint32_t bk = 2 * gbase + (slot & (2 * agg - 1));
    if (has) L.bucket[bk] = tid;
    __syncthreads();
    const uint32_t leader = has ? L.bucket[bk] : tid;
    const bool member = has && L.slot[leader] == slot;
    if (member) {
        lds_add(&L.acc[0][leader], q0);
        lds_add(&L.acc[1][leader], q1);
        lds_add(&L.acc[2][leader], q2);
        atomicAdd(&L.cnt[leader], 1u);
    }
    __syncthreads();
    if (member && leader == tid) {
        accumulate(t, slot, L.cnt[tid], lds_value(&L.acc[0][tid], q0), lds_value(&L.acc[1][tid], q0),
                   lds_value(&L.acc[2][tid], q0));
    } else if (has && !member) {
        accumulate(t, slot, 1, q0, q1, q2);
    }
    __syncthreads();  // the scratch may be reused right after
}

// Temporal values of the occupied cells recorded in occupancy word j of
// Changes of resolution across frames (Section 3.4.2) for a key absent from
// `prev`: its parent (level + 1, cell coordinates floor-divided by 2), whose
// value is distributed to it with an eighth of the parent's samples (in
// integration a parent with fewer than 8 is not used), else its 8 children
// (level - 1, coordinates 2x~ + 0 or 1 per axis), added up: the sum of their
// counts and their count-weighted mean, accumulated in double in the order
// j = dx + 2 dy + 4 dz.  A candidate whose home slot is empty in prev's
// occupancy bitmap is absent without a read of the slot.  Returns whether
// one was found, with its value and count in old.
template <bool kIntegrate>
__device__ __forceinline__ bool find_across_levels(const Tab &prev, uint64_t K, float4 &old) {
    int x[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = (int)((K >> (17 * c)) & 0x1ffffu) - 65536;
    const int lp = (int)((K >> 51) & 31u) - 16;
    const uint64_t code = K >> 56;
    // the parent's and the 8 children's keys, and their home slots' occupancy
    // bits, all loaded before any is used
    uint64_t cand[9];
    bool ok[9];
    ok[0] = lp + 1 <= kLevelMax;
    cand[0] = (code << 56) | ((uint64_t)(uint32_t)(lp + 17) << 51);
#pragma unroll
    for (int c = 0; c < 3; ++c) cand[0] |= (uint64_t)(uint32_t)((x[c] >> 1) + 65536) << (17 * c);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        cand[1 + d] = (code << 56) | ((uint64_t)(uint32_t)(lp + 15) << 51);
        ok[1 + d] = lp - 1 >= kLevelMin;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int y = 2 * x[c] + ((d >> c) & 1);
            ok[1 + d] = ok[1 + d] && y > -65536 && y < 65536;
            cand[1 + d] |= (uint64_t)(uint32_t)(y + 65536) << (17 * c);
        }
    }
    uint32_t home[9], word[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        home[q] = ok[q] ? home_of(cand[q], prev.mask) : 0u;
        word[q] = ok[q] ? prev.occ[home[q] >> 5] : 0u;
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) ok[q] = ok[q] && ((word[q] >> (home[q] & 31)) & 1u);
    if (ok[0]) {
        const uint32_t s = find_exact(prev, cand[0], fingerprint_of(cand[0]));
        if (s != kNoSlot) {
            const float4 v = prev.blend_at(s);
            const uint32_t n = (uint32_t)v.w / 8;
            if (!kIntegrate || n >= 1) {
                old = make_float4(v.x, v.y, v.z, (float)n);
                return true;
            }
        }
    }
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    uint32_t n = 0;
    for (int d = 0; d < 8; ++d) {
        if (!ok[1 + d]) continue;
        const uint32_t s = find_exact(prev, cand[1 + d], fingerprint_of(cand[1 + d]));
        if (s == kNoSlot) continue;
        const float4 v = prev.blend_at(s);
        const uint32_t w = (uint32_t)v.w;
        n += w;
        a0 += (double)w * (double)v.x;
        a1 += (double)w * (double)v.y;
        a2 += (double)w * (double)v.z;
    }
    if (n) {
        old = make_float4((float)(a0 / (double)n), (float)(a1 / (double)n), (float)(a2 / (double)n), (float)n);
        return true;
    }
    return false;
}

// The temporal values of kTB cells of cur: slots s (has: in use), keys,
// fingerprints fp, this frame's averages v and counts cnt, stored counts
// keep.  Each key is searched in prev (fingerprint probe confirmed by the
// stored key) and, where found, blended by the moving average or by
// integration (kIntegrate; keep then becomes min(N_old + N_new, cap)); the
// values are stored in cur's records.  Returns the keys found in prev.
template <bool kHasPrev, bool kIntegrate, int kTB, bool kLevels>
__device__ __forceinline__ uint32_t blend_cells(const Tab &cur, const Tab &prev, const uint32_t (&s)[kTB],
                                                const bool (&has)[kTB], const uint64_t (&key)[kTB],
                                                const uint32_t (&fp)[kTB], float (&v)[kTB][3],
                                                const uint32_t (&cnt)[kTB], uint32_t (&keep)[kTB], float alpha,
                                                float beta, uint32_t cap) {
    uint32_t hits = 0;
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
            for (int k = 0; k < kTB; ++k) pf[k] = active[k] ? prev.cell_at(p[k]).fp : 0u;
#pragma unroll
            for (int k = 0; k < kTB; ++k) {
                pk[k] = 0;
                if (active[k] && pf[k] == fp[k]) pk[k] = prev.key_at(p[k]);
            }
#pragma unroll
            for (int k = 0; k < kTB; ++k) {
                if (!active[k]) continue;
                if (pf[k] == 0) {
                    active[k] = false;  // empty slot: not in prev
                } else if (pf[k] == fp[k] && pk[k] == key[k]) {
                    active[k] = false;
                    found[k] = true;
                } else {
                    p[k] = (p[k] + 1) & prev.mask;
                }
            }
        }
        float4 old[kTB];
        bool use[kTB];
#pragma unroll
        for (int k = 0; k < kTB; ++k) {
            if (found[k]) old[k] = prev.blend_at(p[k]);
            use[k] = found[k];
        }
        if constexpr (kLevels) {
            for (int k = 0; k < kTB; ++k)
                if (has[k] && !found[k]) use[k] = find_across_levels<kIntegrate>(prev, key[k], old[k]);
        }
#pragma unroll
        for (int k = 0; k < kTB; ++k) {
            if (!use[k]) continue;
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
            if (found[k]) ++hits;
        }
    }
#pragma unroll
    for (int k = 0; k < kTB; ++k)
        if (has[k]) cur.blend_at(s[k]) = make_float4(v[k][0], v[k][1], v[k][2], (float)keep[k]);
    return hits;
}

// The temporal blend of the occupied cells of bitmap word j of `cur`
// (Section 3.4.1), restricted to the bits of `part`; returns how many found
// their key in `prev`.  The word's cells are taken kTB at a time, and each
// step of their lookups in the previous table (cell and key, fingerprint
// probe, key check, old value) is issued for all of them before any result
// is used (blend_cells).  kIntegrate: temporal
// integration, alpha = N_old / (N_old + N_new) per cell with the stored count
// kept at most `cap`; else the moving average with a fixed alpha (the stored
// count is this frame's).
// kLevels: a key absent from prev is searched one level coarser and finer
// (find_across_levels); hits still count exact keys only.
template <bool kHasPrev, bool kIntegrate, int kTB = 4, bool kLevels = false>  // kTB: cells looked up together
__device__ __forceinline__ uint32_t temporal_word(const Tab &cur, const Tab &prev, uint32_t j, float alpha,
                                                  float beta, uint32_t cap, uint32_t part = 0xffffffffu) {
    uint32_t hits = 0;
    uint32_t w = cur.occ[j] & part;  // the slots of the word this lane takes
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
                lo[k] = cur.words_at(s[k])[0];
                hi[k] = cur.words_at(s[k])[1];
                if constexpr (kHasPrev) key[k] = cur.key_at(s[k]);
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
        uint32_t fp[kTB];
#pragma unroll
        for (int k = 0; k < kTB; ++k) fp[k] = has[k] ? lo[k].x : 0u;
        hits += blend_cells<kHasPrev, kIntegrate, kTB, kLevels>(cur, prev, s, has, key, fp, v, cnt, keep, alpha, beta,
                                                                cap);
    }
    return hits;
}

// The value a vertex's lookup returns: its cell's temporal value (blend)
// or average, with the count in w, or its own contribution when it has no
// slot (then w is 0).
__device__ __forceinline__ float4 lookup_value(const Tab &t, uint32_t slot, uint32_t i, const float *r, const float *g,
                                               const float *b, bool blend) {
    if (slot == kNoSlot) return make_float4(r[i], g[i], b[i], 0.0f);
    if (blend) return t.blend_at(slot);
    const pf_cell c = t.cell_at(slot);
    return make_float4(t.average(c, 0), t.average(c, 1), t.average(c, 2), (float)c.count);
}

// Lookup for one vertex: writes its filtered contribution (or its own when
// unfiltered) and count.
template <bool kBlend>
__device__ __forceinline__ void query_vertex(const Tab &t, uint32_t slot, uint32_t i, const float *r, const float *g,
                                             const float *b, float *ro, float *go, float *bo, uint32_t *count_out,
                                             bool inplace) {
    if (slot == kNoSlot) {
        if (!inplace) {
            ro[i] = r[i];
            go[i] = g[i];
            bo[i] = b[i];
        }
        if (count_out) count_out[i] = 0;
        return;
    }
    float a0, a1, a2;
    uint32_t cnt;
    if constexpr (kBlend) {
        const float4 v = t.blend_at(slot);
        a0 = v.x;
        a1 = v.y;
        a2 = v.z;
        cnt = (uint32_t)v.w;
    } else {
        const pf_cell c = t.cell_at(slot);
        cnt = c.count;
        a0 = t.average(c, 0);
        a1 = t.average(c, 1);
        a2 = t.average(c, 2);
    }
    ro[i] = a0;
    go[i] = a1;
    bo[i] = a2;
    if (count_out) count_out[i] = cnt;
}

}  // namespace pfk
