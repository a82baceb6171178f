// Many views in one persistent launch on gfx950.  A cooperative grid of
// resident workgroups walks four phases -- clear, keys + insert, reduce with
// the temporal blend, lookup -- separated by grid-wide barriers.  Within a
// phase the work items of all views (chunks of bitmap words, windows of
// vertices, bins of slots) are dealt to the workgroups round-robin, so small
// and large views share the whole chip.  As in the single-view binned
// insert, the insert adds nothing to the cells: each group of vertices that
// share a key in a window claims its cell and writes one record {slot,
// count, sums} into its bin's bucket (one part per XCD, position by one
// device atomic add); the reduce phase gives every bin of every view to one
// workgroup, which sums the bin's records in LDS, adds them to its cells
// with plain loads and stores, and blends the cells with the previous
// frame's values.  The per-vertex and per-cell arithmetic is that of the
// single-view kernels (pf_ops.h).
#include "pf_grid.h"
#include "pf_kernels.h"
#include "pf_merge.h"
#include "pf_ops.h"

namespace pfk {

namespace views {

using grid::Barrier;
using grid::grid_barrier;
using grid::kCounterStride;
using grid::kSubCounters;
using grid::poll;

constexpr int kIters = 8;            // block-sized steps per work item
constexpr uint32_t kParts = 8;       // bucket parts per bin: one per XCD
__device__ __forceinline__ Tab to_tab(const pf_table &t) {
    Tab k;
    k.rec = reinterpret_cast<unsigned char *>(t.cell);
    k.occ = t.occ;
    k.stats = reinterpret_cast<unsigned long long *>(t.stats);
    k.mask = (uint32_t)((1ull << t.log2_slots) - 1);
    k.max_probe = t.max_probe;
    k.frac_bits = t.frac_bits;
    k.fsum = 0;  // float tables are rejected on the host
    return k;
}

// LDS merge table of the insert phase: a window of agg_width consecutive
// vertices (block .. kIters * block) merges into at most min(agg_width,
// 4 * block, 1536) entries (the table stays in static LDS and small
// workgroups keep their residency); a vertex that finds no room goes alone.
template <int B>
constexpr uint32_t kMergeCap = 4 * B < 1536 ? 4 * B : 1536;
template <int B>
constexpr uint32_t kEntries = (kMergeCap<B> + B - 1) / B;  // merge-table entries per lane
// Bins of the reduce phase: 4 * block slots (at most 2048), whose count and
// sums the workgroup holds in LDS (no more than the merge table takes).
template <int B>
constexpr uint32_t kBinSlots = 4 * B < 2048 ? 4 * B : 2048;
template <int B>
constexpr uint32_t kBinShift = B >= 512 ? 11u : (uint32_t)__builtin_ctz(4 * B);

template <int B>
struct Lds {
    union {
        struct {
            unsigned long long key[kMergeCap<B>];
            unsigned long long s0[kMergeCap<B>], s1[kMergeCap<B>], s2[kMergeCap<B>];
            uint32_t cnt[kMergeCap<B>];  // count, then the group's slot
        } m;
        struct {
            unsigned long long s0[kBinSlots<B>], s1[kBinSlots<B>], s2[kBinSlots<B>];  // s0 then holds the cell list
            uint32_t cnt[kBinSlots<B>];
        } r;
    };
    uint32_t first[5][PF_MAX_VIEWS + 1];  // per item kind: first global item of each view
    uint32_t seg[kParts + 1];
    uint32_t spilled[2048 / 32];  // occupancy bits that spilled groups set, per bin
    uint32_t hits, nlist;
};

template <int B>
__device__ __forceinline__ void item_of(const Lds<B> &L, int phase, uint32_t nviews, uint32_t it, uint32_t &v,
                                        uint32_t &local) {
    v = 0;
    while (v + 1 < nviews && it >= L.first[phase][v + 1]) ++v;
    local = it - L.first[phase][v];
}

// Key, flags and fixed-point contribution of vertex i of a view (masked
// vertices read nothing more than their valid byte).
__device__ __forceinline__ uint8_t view_vertex(const pf_view &d, const Tab &t, float inv_s, uint32_t i, uint64_t &key,
                                               int64_t &q0, int64_t &q1, int64_t &q2) {
    key = 0;
    q0 = q1 = q2 = 0;
    if (d.valid != nullptr && d.valid[i] == 0) return PF_V_INVALID;
    const float x[3] = {d.px[i], d.py[i], d.pz[i]};
    const float nr[3] = {d.nx[i], d.ny[i], d.nz[i]};
    uint32_t fp, home;
    const PcgJump jp(d.kp.seed, d.kp.idx_base);
    uint8_t fl = vertex_key(x, nr, true, d.kp.cam, d.kp.s, inv_s, jp, i, t.mask, key, fp, home);
    if (fl == 0) fl = fixed_point(d.r[i], d.g[i], d.b[i], t.frac_bits, q0, q1, q2);
    return fl;
}

// Empties the cells of bitmap word j of t and the word.
__device__ __forceinline__ void clear_word(const Tab &t, uint32_t j) {
    uint32_t w = t.occ[j];
    if (w) t.occ[j] = 0;
    while (w) {
        const uint32_t b = __builtin_ctz(w);
        w &= w - 1;
        uint4 *c = t.words_at(j * 32 + b);
        c[0] = make_uint4(0, 0, 0, 0);
        c[1] = make_uint4(0, 0, 0, 0);
    }
}

template <int B>
__device__ __forceinline__ uint32_t bin_shift_of(uint32_t log2_slots) {
    return kBinShift<B> < log2_slots ? kBinShift<B> : log2_slots;
}

// Probe / claim like find_or_claim, without the occupancy bit (the reduce
// phase sets the bits of the cells it receives records for), from probe d0
// at slot s onwards.
__device__ __forceinline__ uint32_t claim_cell_from(const Tab &t, uint64_t key, uint32_t f, uint32_t s, uint32_t d0) {
    for (uint32_t d = d0; d < t.max_probe; ++d) {
        uint32_t *pfp = &t.cell_at(s).fp;
        uint32_t cur = load_fp_probe(pfp);
        if (cur == 0) {
            uint32_t expected = 0;
            if (__hip_atomic_compare_exchange_strong(pfp, &expected, f, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                t.key_at(s) = key;
                return s;
            }
            cur = expected;
        }
        if (cur == f) return s;
        s = (s + 1) & t.mask;
    }
    return kNoSlot;
}

__device__ __forceinline__ uint32_t claim_cell(const Tab &t, uint64_t key) {
    return claim_cell_from(t, key, fingerprint_of(key), home_of(key, t.mask), 0);
}

// One group's record {slot, count, sums} into its bin's bucket part for this
// workgroup's XCD; a full part sends the group to its cell by device
// atomics instead, and sets the cell's occupancy bit.
// pos: the record's position in its part, taken from the part's count.
__device__ __forceinline__ void put_record(const ViewDev &vd, const Tab &t, uint32_t bin_shift, uint32_t part,
                                           uint32_t pos, uint32_t s, uint32_t count, uint64_t s0, uint64_t s1,
                                           uint64_t s2) {
    const size_t at = (size_t)(s >> bin_shift) * kParts + part;
    if (pos < vd.part_cap) {
        uint4 *w = vd.rec + 2 * (at * vd.part_cap + pos);
        w[0] = make_uint4(s, count, (uint32_t)s0, (uint32_t)(s0 >> 32));
        w[1] = make_uint4((uint32_t)s1, (uint32_t)(s1 >> 32), (uint32_t)s2, (uint32_t)(s2 >> 32));
    } else {
        accumulate(t, s, count, (int64_t)s0, (int64_t)s1, (int64_t)s2);
        __hip_atomic_fetch_or(&t.occ[s >> 5], 1u << (s & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ void put_group(const ViewDev &vd, const Tab &t, uint32_t bin_shift, uint32_t part,
                                          uint32_t s, uint32_t count, uint64_t s0, uint64_t s1, uint64_t s2) {
    const uint32_t pos = __hip_atomic_fetch_add(&vd.cnt[(size_t)(s >> bin_shift) * kParts + part], 1u,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    put_record(vd, t, bin_shift, part, pos, s, count, s0, s1, s2);
}

// At least kWavesPerSimd waves of this kernel fit a SIMD (the compiler
// keeps the registers within that), which bounds the resident workgroups
// from below independently of the occupancy query.  1024-lane workgroups
// ask for 8, so that two of them (32 waves) share a compute unit as the
// single-view insert's do.
template <int B>
constexpr int kWavesPerSimd = B >= 1024 ? 8 : 4;

template <int B>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd<B>))) void views_kernel(
    const ViewDev *__restrict__ views, uint32_t nviews, uint32_t agg, Barrier bar) {
    __shared__ Lds<B> L;
    constexpr uint32_t kItem = (uint32_t)B * kIters;
    // work items per view and kind: 0 clear cur (B bitmap words and bucket
    // counts), 1 keys + insert (8 x B vertices), 2 reduce and temporal (one
    // bin), 3 clear prev (B bitmap words), 4 lookup (8 x B vertices); kinds
    // 3 and 4 share the last phase
    if (threadIdx.x == 0) {
        uint32_t acc[5] = {0, 0, 0, 0, 0};
        for (uint32_t v = 0; v < nviews; ++v) {
            const pf_view &d = views[v].d;
            const uint32_t slots = 1u << d.cur.log2_slots;
            const uint32_t words = (slots + 31) / 32;
            const uint32_t counts = views[v].nbins * kParts;
            const uint32_t zero = words > counts ? words : counts;
            const uint32_t items[5] = {(zero + B - 1) / B, (d.n + kItem - 1) / kItem, views[v].nbins,
                                       d.prev.cell ? (words + B - 1) / B : 0u, (d.n + kItem - 1) / kItem};
            for (int p = 0; p < 5; ++p) {
                L.first[p][v] = acc[p];
                acc[p] += items[p];
            }
        }
        for (int p = 0; p < 5; ++p) L.first[p][nviews] = acc[p];
    }
    // block 0 stamps the start and the end of every phase (wall clock, as
    // 64-bit values in status words 4..13) for the caller's diagnostics
    auto stamp = [&](int k) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const uint64_t w = wall_clock64();
            bar.status[4 + 2 * k] = (uint32_t)w;
            bar.status[5 + 2 * k] = (uint32_t)(w >> 32);
        }
    };
    if (blockIdx.x == 0 && threadIdx.x == 0) bar.status[1] = gridDim.x;
    stamp(0);
    __syncthreads();
    const uint32_t G = gridDim.x;
    const uint32_t part = blockIdx.x % kParts;  // workgroups are dealt to the XCDs in turn

    // ---- phase 0: clear the current tables (nothing to do where the last
    // launch emptied them) and the bucket counts
    for (uint32_t it = blockIdx.x; it < L.first[0][nviews]; it += G) {
        uint32_t v, local;
        item_of(L, 0, nviews, it, v, local);
        const ViewDev &vd = views[v];
        const Tab t = to_tab(vd.d.cur);
        const uint32_t j = local * B + threadIdx.x;  // one bitmap word and one count per lane
        if (j < t.nwords()) clear_word(t, j);
        if (j < vd.nbins * kParts) vd.cnt[j] = 0;
        if (local == 0)
            for (uint32_t k = threadIdx.x; k < PF_STATS_LEN; k += B) t.stats[k] = 0;
    }
    if (!grid_barrier(bar, 1)) return;
    stamp(1);

    // ---- phase 1: keys and insertion.  agg == 0: one claim and one set of
    // device atomics per vertex.  Otherwise each window of agg consecutive
    // vertices (a power of two, block <= agg <= kIters * block) merges by key
    // in LDS, then every group claims its cell once and writes one record to
    // its bin's bucket.
    const uint32_t kCap = agg < kMergeCap<B> ? agg : kMergeCap<B>;
    const uint32_t per = agg / B;  // vertices per lane and window (1, 2, 4 or 8)
    for (uint32_t it = blockIdx.x; it < L.first[1][nviews]; it += G) {
        uint32_t v, local;
        item_of(L, 1, nviews, it, v, local);
        const ViewDev &vd = views[v];
        const pf_view &d = vd.d;
        const Tab t = to_tab(d.cur);
        const float inv_s = 1.0f / d.kp.s;
        const uint32_t bshift = bin_shift_of<B>(d.cur.log2_slots);
        if (agg == 0) {
            for (int k = 0; k < kIters; ++k) {
                const uint32_t i = local * kItem + k * B + threadIdx.x;
                if (i >= d.n) break;
                uint64_t key;
                int64_t q0 = 0, q1 = 0, q2 = 0;
                uint32_t slot = kNoSlot;
                uint8_t fl = view_vertex(d, t, inv_s, i, key, q0, q1, q2);
                if (fl == 0) {
                    slot = find_or_claim(t, key);
                    if (slot == kNoSlot) {
                        fl = PF_V_OVERFLOW;
                        add_u64(&t.stats[PF_STAT_PART_OVF + (blockIdx.x & 15)], 1ull);
                    } else {
                        accumulate(t, slot, 1, q0, q1, q2);
                    }
                }
                if (d.key) d.key[i] = key;
                d.vflags[i] = fl;
                d.slot[i] = slot;
            }
            continue;
        }
        for (uint32_t sub = 0; sub < (uint32_t)kIters / per; ++sub) {
            const uint32_t base = local * kItem + sub * agg;
            if (base >= d.n) break;  // uniform across the workgroup
            for (uint32_t j = threadIdx.x; j < kCap; j += B) {
                L.m.key[j] = kEmpty;
                L.m.s0[j] = 0;
                L.m.s1[j] = 0;
                L.m.s2[j] = 0;
                L.m.cnt[j] = 0;
            }
            __syncthreads();
            // a lane keeps only its vertices' flags and LDS entries across
            // the barriers; the rare vertex that found no room rebuilds its
            // key and contribution
            uint64_t fv = 0;          // 8 bits per vertex
            uint64_t ev[2] = {0, 0};  // 16 bits per vertex (4 per word), 0xffff = no room
#pragma unroll 1
            for (uint32_t u = 0; u < per; ++u) {
                const uint32_t i = base + u * B + threadIdx.x;
                uint64_t k = 0;
                int64_t q0 = 0, q1 = 0, q2 = 0;
                uint8_t f = PF_V_INVALID;
                if (i < d.n) f = view_vertex(d, t, inv_s, i, k, q0, q1, q2);
                if (d.key && i < d.n) d.key[i] = k;
                const int e =
                    merge_into_lds<false>(L.m.key, L.m.s0, L.m.s1, L.m.s2, L.m.cnt, kCap, f == 0, k, q0, q1, q2);
                fv |= (uint64_t)f << (8 * u);
                const uint64_t eb = (uint64_t)(uint16_t)e << (16 * (u & 3));
                if (u < 4)
                    ev[0] |= eb;
                else
                    ev[1] |= eb;
            }
            __syncthreads();
            // one claim and one record per group; a lane's entries issue
            // their home-slot loads, then their compare-and-swaps on empty
            // home slots, then their bucket positions, before any result is
            // used
            uint64_t gk[kEntries<B>];
            uint32_t fs[kEntries<B>], ff[kEntries<B>], fc[kEntries<B>], sl[kEntries<B>], pos[kEntries<B>];
            bool won[kEntries<B>];
#pragma unroll
            for (uint32_t e = 0; e < kEntries<B>; ++e) {
                const uint32_t j = e * B + threadIdx.x;
                gk[e] = j < kCap ? L.m.key[j] : kEmpty;
                fs[e] = ff[e] = fc[e] = 0;
                if (gk[e] != kEmpty) {
                    fs[e] = home_of(gk[e], t.mask);
                    ff[e] = fingerprint_of(gk[e]);
                    fc[e] = load_fp_probe(&t.cell_at(fs[e]).fp);
                }
            }
#pragma unroll
            for (uint32_t e = 0; e < kEntries<B>; ++e) {
                won[e] = false;
                if (gk[e] != kEmpty && fc[e] == 0) {
                    uint32_t expected = 0;
                    won[e] = __hip_atomic_compare_exchange_strong(&t.cell_at(fs[e]).fp, &expected, ff[e],
                                                                  __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_AGENT);
                    fc[e] = won[e] ? ff[e] : expected;
                }
            }
#pragma unroll
            for (uint32_t e = 0; e < kEntries<B>; ++e) {
                sl[e] = kNoSlot;
                pos[e] = 0;
                if (gk[e] == kEmpty) continue;
                if (won[e]) t.key_at(fs[e]) = gk[e];
                // the home slot holds another key: probe on from the next
                sl[e] = fc[e] == ff[e] ? fs[e] : claim_cell_from(t, gk[e], ff[e], (fs[e] + 1) & t.mask, 1);
                if (sl[e] != kNoSlot)
                    pos[e] = __hip_atomic_fetch_add(&vd.cnt[(size_t)(sl[e] >> bshift) * kParts + part], 1u,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
#pragma unroll
            for (uint32_t e = 0; e < kEntries<B>; ++e) {
                const uint32_t j = e * B + threadIdx.x;
                if (gk[e] == kEmpty) continue;
                const uint32_t c = L.m.cnt[j];
                if (sl[e] != kNoSlot)
                    put_record(vd, t, bshift, part, pos[e], sl[e], c, L.m.s0[j], L.m.s1[j], L.m.s2[j]);
                else
                    add_u64(&t.stats[PF_STAT_PART_OVF + (blockIdx.x & 15)], (unsigned long long)c);
                L.m.cnt[j] = sl[e];
            }
            __syncthreads();
#pragma unroll 1
            for (uint32_t u = 0; u < per; ++u) {
                const uint32_t i = base + u * B + threadIdx.x;
                if (i >= d.n) continue;
                uint8_t fl = (uint8_t)(fv >> (8 * u));
                const uint32_t e = (uint32_t)((u < 4 ? ev[0] : ev[1]) >> (16 * (u & 3))) & 0xffffu;
                uint32_t slot = kNoSlot;
                if (fl == 0) {
                    if (e != 0xffffu) {
                        slot = L.m.cnt[e];
                    } else {  // no room in the LDS table: on its own
                        uint64_t k;
                        int64_t q0, q1, q2;
                        view_vertex(d, t, inv_s, i, k, q0, q1, q2);
                        slot = claim_cell(t, k);
                        if (slot != kNoSlot)
                            put_group(vd, t, bshift, part, slot, 1u, (uint64_t)q0, (uint64_t)q1, (uint64_t)q2);
                        else
                            add_u64(&t.stats[PF_STAT_PART_OVF + (blockIdx.x & 15)], 1ull);
                    }
                    if (slot == kNoSlot) fl = PF_V_OVERFLOW;
                }
                d.vflags[i] = fl;
                d.slot[i] = slot;
            }
            __syncthreads();  // the table is cleared for the next window
        }
    }
    if (!grid_barrier(bar, 2)) return;
    stamp(2);

    // ---- phase 2: per bin, the records summed in LDS and added to the
    // cells by the workgroup that owns them, then the temporal values of the
    // bin's cells (claimed cells have their occupancy bits set)
    for (uint32_t it = blockIdx.x; it < L.first[2][nviews]; it += G) {
        uint32_t v, local;
        item_of(L, 2, nviews, it, v, local);
        const ViewDev &vd = views[v];
        const pf_view &d = vd.d;
        const Tab cur = to_tab(d.cur);
        const uint32_t bshift = bin_shift_of<B>(d.cur.log2_slots);
        const uint32_t bslots = 1u << bshift;
        const uint32_t base = local << bshift;
        for (uint32_t k = threadIdx.x; k < bslots; k += B) {
            L.r.s0[k] = 0;
            L.r.s1[k] = 0;
            L.r.s2[k] = 0;
            L.r.cnt[k] = 0;
        }
        if (threadIdx.x == 0) {
            uint32_t acc = 0;
            for (uint32_t x = 0; x < kParts; ++x) {
                L.seg[x] = acc;
                const uint32_t c = vd.cnt[(size_t)local * kParts + x];
                acc += c < vd.part_cap ? c : vd.part_cap;
            }
            L.seg[kParts] = acc;
            L.hits = 0;
            L.nlist = 0;
        }
        // before this phase only spilled groups and per-vertex atomics
        // (agg_width 0) set bits of the cleared table
        for (uint32_t w = threadIdx.x; w < (bslots + 31) / 32; w += B) L.spilled[w] = cur.occ[(base >> 5) + w];
        __syncthreads();
        const uint4 *in = vd.rec + 2 * (size_t)local * kParts * vd.part_cap;
        const uint32_t j1 = L.seg[kParts];
        for (uint32_t j = threadIdx.x; j < j1; j += B) {
            uint32_t x = 0;
#pragma unroll
            for (uint32_t y = 1; y < kParts; ++y) x = j >= L.seg[y] ? y : x;
            const size_t at = (size_t)x * vd.part_cap + (j - L.seg[x]);
            const uint4 lo = in[2 * at], hi = in[2 * at + 1];
            const uint32_t loc = lo.x - base;
            atomicAdd(&L.r.cnt[loc], lo.y);
            atomicAdd(&L.r.s0[loc], (unsigned long long)lo.z | (unsigned long long)lo.w << 32);
            atomicAdd(&L.r.s1[loc], (unsigned long long)hi.x | (unsigned long long)hi.y << 32);
            atomicAdd(&L.r.s2[loc], (unsigned long long)hi.z | (unsigned long long)hi.w << 32);
        }
        __syncthreads();
        for (uint32_t k0 = 0; k0 < bslots; k0 += B) {  // uniform: every lane reaches the ballot
            const uint32_t k = k0 + threadIdx.x;
            const uint32_t c = k < bslots ? L.r.cnt[k] : 0u;
            if (c) {
                uint4 *cells = cur.words_at(base + k);
                const uint4 lo = cells[0], hi = cells[1];
                const uint64_t s0 = ((uint64_t)lo.z | (uint64_t)lo.w << 32) + L.r.s0[k];
                const uint64_t s1 = ((uint64_t)hi.x | (uint64_t)hi.y << 32) + L.r.s1[k];
                const uint64_t s2 = ((uint64_t)hi.z | (uint64_t)hi.w << 32) + L.r.s2[k];
                cells[0] = make_uint4(lo.x, lo.y + c, (uint32_t)s0, (uint32_t)(s0 >> 32));
                cells[1] = make_uint4((uint32_t)s1, (uint32_t)(s1 >> 32), (uint32_t)s2, (uint32_t)(s2 >> 32));
            }
            // occupancy: a wavefront's 64 consecutive slots are two bitmap
            // words of this bin (bins hold >= 256 slots) or, in a table of 16
            // slots, half of one
            const uint64_t m = __ballot(c != 0);
            if ((threadIdx.x & 63) == 0 && m) {
                const uint32_t w = (base + k) >> 5;
                if ((uint32_t)m) cur.occ[w] |= (uint32_t)m;
                if (m >> 32) cur.occ[w + 1] |= (uint32_t)(m >> 32);
            }
        }
        if (d.temporal) {
            __syncthreads();  // the sums are no longer read: their space holds the list of the bin's cells
            uint32_t *list = reinterpret_cast<uint32_t *>(L.r.s0);
            for (uint32_t k = threadIdx.x; k < bslots; k += B)
                if (L.r.cnt[k] || ((L.spilled[k >> 5] >> (k & 31)) & 1u)) list[atomicAdd(&L.nlist, 1u)] = k;
            __syncthreads();
            const bool has_prev = d.prev.cell != nullptr;
            const Tab prev = has_prev ? to_tab(d.prev) : cur;
            const float alpha = d.alpha_old, beta = 1.0f - d.alpha_old;
            uint32_t hits = 0;
            for (uint32_t q = threadIdx.x; q < L.nlist; q += B) {
                const uint32_t sl[1] = {base + list[q]};
                const uint4 *w4 = cur.words_at(sl[0]);  // written above by this workgroup
                const uint4 lo = w4[0], hi = w4[1], kw = w4[2];
                pf_cell cl;
                cl.fp = lo.x;
                cl.count = lo.y;
                cl.sum[0] = (int64_t)((uint64_t)lo.z | (uint64_t)lo.w << 32);
                cl.sum[1] = (int64_t)((uint64_t)hi.x | (uint64_t)hi.y << 32);
                cl.sum[2] = (int64_t)((uint64_t)hi.z | (uint64_t)hi.w << 32);
                const bool has[1] = {true};
                const uint64_t key[1] = {(uint64_t)kw.x | (uint64_t)kw.y << 32};
                const uint32_t fp[1] = {cl.fp}, n[1] = {cl.count};
                uint32_t keep[1] = {cl.count};
                float val[1][3] = {{cur.average(cl, 0), cur.average(cl, 1), cur.average(cl, 2)}};
                if (has_prev)
                    hits += blend_cells<true, false, 1, false>(cur, prev, sl, has, key, fp, val, n, keep, alpha, beta,
                                                               0u);
                else
                    blend_cells<false, false, 1, false>(cur, prev, sl, has, key, fp, val, n, keep, alpha, beta, 0u);
            }
            if (has_prev) {
                if (hits) atomicAdd(&L.hits, hits);
                __syncthreads();
                if (threadIdx.x == 0 && L.hits) add_u64(&cur.stats[PF_STAT_PART_HIT + (blockIdx.x & 31)], L.hits);
            }
        }
        __syncthreads();  // the LDS is cleared for the next bin
    }
    if (!grid_barrier(bar, 3)) return;
    stamp(3);

    // ---- phase 3: empty the previous tables (read for the last time by the
    // temporal blend), then look up every vertex; the clear's items come
    // first, so its scattered stores overlap the lookup's gathers
    const uint32_t n_clear = L.first[3][nviews];
    for (uint32_t it = blockIdx.x; it < n_clear + L.first[4][nviews]; it += G) {
        uint32_t v, local;
        if (it < n_clear) {
            item_of(L, 3, nviews, it, v, local);
            const Tab t = to_tab(views[v].d.prev);
            const uint32_t j = local * B + threadIdx.x;
            if (j < t.nwords()) clear_word(t, j);
            continue;
        }
        item_of(L, 4, nviews, it - n_clear, v, local);
        const pf_view &d = views[v].d;
        const Tab t = to_tab(d.cur);
        // four vertices at a time: their slots (kNoSlot for flagged vertices),
        // then every value they read, then the stores, so the loads of the
        // four are in flight together
        for (int k0 = 0; k0 < kIters; k0 += 4) {
            uint32_t slot[4];
            float4 val[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = local * kItem + (k0 + u) * B + threadIdx.x;
                slot[u] = i < d.n ? d.slot[i] : kNoSlot;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = local * kItem + (k0 + u) * B + threadIdx.x;
                if (i >= d.n) continue;
                val[u] = lookup_value(t, slot[u], i, d.r, d.g, d.b, d.temporal != 0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t i = local * kItem + (k0 + u) * B + threadIdx.x;
                if (i >= d.n) continue;
                d.r_out[i] = val[u].x;
                d.g_out[i] = val[u].y;
                d.b_out[i] = val[u].z;
                if (d.count_out) d.count_out[i] = slot[u] == kNoSlot ? 0u : (uint32_t)val[u].w;
            }
        }
    }
    // the lookup has no barrier after it: block 0 stamps its own end
    stamp(4);
}

__global__ void views_reset_kernel(uint32_t *ws, uint32_t words) {
    for (uint32_t j = threadIdx.x; j < words; j += blockDim.x) ws[j] = 0;
}

// Workspace layout for workgroups of B threads: barrier counters, the device
// copy of the descriptors, then per view its bucket counts and records.
struct Layout {
    size_t desc, bytes;
    size_t cnt[PF_MAX_VIEWS], rec[PF_MAX_VIEWS];
    uint32_t nbins[PF_MAX_VIEWS], part_cap[PF_MAX_VIEWS];
};

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

Layout layout(const uint64_t *n, const uint32_t *log2_slots, uint32_t nviews, uint32_t block) {
    Layout l;
    const uint32_t bs = block >= 512 ? 11u : (uint32_t)__builtin_ctz(4 * block);
    size_t off = align256(sizeof(uint32_t) * kCounterStride * (2 * kSubCounters + 2));
    l.desc = off;
    off += align256(nviews * sizeof(ViewDev));
    for (uint32_t v = 0; v < nviews; ++v) {
        const uint32_t shift = bs < log2_slots[v] ? bs : log2_slots[v];
        l.nbins[v] = 1u << (log2_slots[v] - shift);
        const uint64_t nparts = (uint64_t)l.nbins[v] * kParts;
        // twice one record per vertex over the parts
        const uint64_t cap = (2 * (n[v] ? n[v] : 1) + nparts - 1) / nparts;
        l.part_cap[v] = (uint32_t)cap;
        l.cnt[v] = off;
        off += align256(nparts * sizeof(uint32_t));
        l.rec[v] = off;
        off += align256(nparts * cap * 32);
    }
    l.bytes = off + 256;
    return l;
}

template <int B>
hipError_t launch_b(const ViewDev *views, uint32_t nviews, uint32_t agg, uint32_t per_cu, uint32_t *ws,
                    hipStream_t st) {
    static int resident = 0;  // workgroups per CU for this block size (queried once)
    static int cus = 0;
    if (resident == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, reinterpret_cast<const void *>(views_kernel<B>), B,
                                                         0);
        if (e != hipSuccess) return e;
        // every workgroup of a cooperative grid must be resident at once: the
        // LDS-bound count is taken as well, with the static LDS rounded up to
        // 2 KB, so that an allocation granularity the occupancy query may not
        // model cannot leave a workgroup waiting for a slot
        int lds_cu = 0;
        e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
        if (e != hipSuccess) return e;
        hipFuncAttributes fa;
        e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(views_kernel<B>));
        if (e != hipSuccess) return e;
        const size_t per_wg = (fa.sharedSizeBytes + 2047) / 2048 * 2048;
        if (per_wg > 0 && lds_cu > 0 && (size_t)resident * per_wg > (size_t)lds_cu)
            resident = (int)((size_t)lds_cu / per_wg);
        // and the register-bound count the compiler guarantees (4 SIMDs)
        const int by_waves = 4 * kWavesPerSimd<B> * 64 / B > 0 ? 4 * kWavesPerSimd<B> * 64 / B : 1;
        if (resident > by_waves) resident = by_waves;
        if (resident < 1) return hipErrorInvalidConfiguration;
    }
    static uint64_t ticks_per_s = 0;
    if (ticks_per_s == 0) {
        int dev = 0, khz = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess) return e;
        ticks_per_s = (uint64_t)(khz > 0 ? khz : 100000) * 1000ull;
    }
    const Barrier bar = grid::barrier_at(ws, 2 * ticks_per_s);  // a phase never takes seconds
    views_reset_kernel<<<1, 256, 0, st>>>(ws, grid::kWords);
    const uint32_t per = (per_cu == 0 || per_cu > (uint32_t)resident) ? (uint32_t)resident : per_cu;
    uint32_t grid = per * (uint32_t)cus;
    void *args[] = {(void *)&views, (void *)&nviews, (void *)&agg, (void *)&bar};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(views_kernel<B>), dim3(grid), dim3(B), args, 0,
                                      st);
}

}  // namespace views

size_t views_workspace_bytes(const uint64_t *n, const uint32_t *log2_slots, uint32_t nviews) {
    size_t most = 0;
    for (uint32_t b = 64; b <= 1024; b *= 2) {
        const size_t x = views::layout(n, log2_slots, nviews, b).bytes;
        most = x > most ? x : most;
    }
    return most;
}

hipError_t launch_views(const pf_view *host_views, uint32_t nviews, uint32_t block, uint32_t agg, uint32_t per_cu,
                        void *workspace, size_t workspace_bytes, hipStream_t st) {
    uint64_t n[PF_MAX_VIEWS];
    uint32_t lg[PF_MAX_VIEWS];
    for (uint32_t v = 0; v < nviews; ++v) {
        n[v] = host_views[v].n;
        lg[v] = host_views[v].cur.log2_slots;
    }
    const views::Layout l = views::layout(n, lg, nviews, block);
    if (l.bytes > workspace_bytes) return hipErrorInvalidValue;
    char *base = reinterpret_cast<char *>(workspace);
    ViewDev desc[PF_MAX_VIEWS];
    for (uint32_t v = 0; v < nviews; ++v) {
        desc[v].d = host_views[v];
        desc[v].cnt = reinterpret_cast<uint32_t *>(base + l.cnt[v]);
        desc[v].rec = reinterpret_cast<uint4 *>(base + l.rec[v]);
        desc[v].nbins = l.nbins[v];
        desc[v].part_cap = l.part_cap[v];
    }
    ViewDev *dev = reinterpret_cast<ViewDev *>(base + l.desc);
    hipError_t e = hipMemcpyAsync(dev, desc, nviews * sizeof(ViewDev), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    uint32_t *ws = reinterpret_cast<uint32_t *>(workspace);
    switch (block) {
        case 64: return views::launch_b<64>(dev, nviews, agg, per_cu, ws, st);
        case 128: return views::launch_b<128>(dev, nviews, agg, per_cu, ws, st);
        case 256: return views::launch_b<256>(dev, nviews, agg, per_cu, ws, st);
        case 512: return views::launch_b<512>(dev, nviews, agg, per_cu, ws, st);
        case 1024: return views::launch_b<1024>(dev, nviews, agg, per_cu, ws, st);
        default: return hipErrorInvalidConfiguration;
    }
}

}  // namespace pfk
