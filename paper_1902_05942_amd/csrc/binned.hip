// Insert-accumulate without device atomics on the cell sums, for gfx950.
//
// Device atomics run at ~24 G/s on MI355X whatever the footprint, and a
// random access of any kind moves a whole cache line, so the cost of the
// insert is the number of per-cell operations it sends to memory.  This path
// sends one per group of vertices that share a key within a chunk of 4096
// consecutive vertices, and no atomic at all for the sums:
//   aggregate  per tile (every ntiles-th chunk): each chunk's vertices are
//              merged by key in an LDS hash table (count and fixed-point
//              sums added with LDS atomics; the LDS serialises the lanes of
//              a coherent run on one entry more cheaply than a wavefront
//              prefix sum over them costs in VALU work, which bounds this
//              kernel); each group then probes / claims its cell once
//              (compare-and-swap on new cells only) and writes one record
//              {slot, count, sums} into its bin's bucket (a bin is a range
//              of slots; a bucket has one part per XCD, so that the records
//              of a cache line are written through one L2), its position
//              taken with one device atomic add; every vertex receives its
//              group's slot
//   reduce     per bin: records summed in LDS, then count and sums added
//              to the cells with plain loads and stores by the workgroup
//              that owns them, occupancy bits set; with a temporal blend
//              (Section 3.4.1) in the same launch, the owner also blends
//              each cell's final average with the previous table's value of
//              its key and stores the temporal value
// A bucket part that is full (never at the workloads' densities: it holds
// twice a vertex's share) takes further groups' counts and sums by device
// atomics on the cell instead, and the group's occupancy bit is set at once.
// Integer sums make the result identical to the atomic insert.
#include <mutex>

#include "pf_kernels.h"
#include "pf_merge.h"
#include "pf_ops.h"

namespace pfk {

namespace binned {

constexpr int kT = 1024;                     // threads of the tile kernels
constexpr uint32_t kPer = 4;                 // vertices per thread and chunk
constexpr uint32_t kChunk = kT * kPer;       // vertices merged in one LDS table
constexpr uint32_t kMaxTiles = 512;          // two workgroups on each of 256 CUs
constexpr uint32_t kLdsBudget = 80 * 1024;   // two 1024-thread workgroups per CU
constexpr uint32_t kFlush = 2;               // LDS entries per thread (entries <= kFlush * kT)
constexpr uint32_t kMaxLog2Slots = 25;
constexpr int kReduceThreads = 1024;  // the bin's LDS sums allow two workgroups per CU

// One staged group: the cell layout with the slot in place of the fingerprint.
struct __align__(16) Rec {
    uint32_t slot, count;
    int64_t s[3];
};
static_assert(sizeof(Rec) == 32, "record is two 16-byte words");

// Inputs of key construction when the insert builds the keys itself.
struct FusedKeys {
    const float *px, *py, *pz, *nx, *ny, *nz;
    const uint8_t *valid;
    KeyArgs a;
    uint64_t *key_out;  // nullable
};

constexpr uint32_t kXcds = 8;  // bucket parts per bin: workgroup w runs on XCD w % 8

struct Plan {
    uint32_t log2_bins, nbins, bin_shift, bin_slots, ntiles, cap, parts, part_cap;
    size_t lds_aggregate, lds_reduce;
    size_t off_cnt, off_rec, bytes;
};

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

Plan make_plan(uint32_t n, uint32_t log2_slots) {
    Plan p;
    // bins of 2048 slots (4096 above 2^24 slots)
    uint32_t lbs = log2_slots > 24 ? 12 : 11;
    if (lbs > log2_slots) lbs = log2_slots;
    p.bin_shift = lbs;
    p.bin_slots = 1u << lbs;
    p.log2_bins = log2_slots - lbs;
    p.nbins = 1u << p.log2_bins;
    // a tile is the set of chunks one workgroup takes (every ntiles-th)
    const uint32_t nchunks = (n + kChunk - 1) / kChunk;
    p.ntiles = nchunks < kMaxTiles ? (nchunks ? nchunks : 1) : kMaxTiles;
    // LDS of aggregate: key 8 B, sums 24 B and count 4 B per entry, four
    // counters, the chunk's list of valid vertices and each vertex's entry
    // (2 B each per vertex); entries take what the budget leaves
    const size_t fixed = 16 + (size_t)kChunk * 4;
    uint32_t cap = (uint32_t)((kLdsBudget - fixed) / 36) / 64 * 64;
    if (cap > kFlush * kT) cap = kFlush * kT;
    p.cap = cap;
    p.lds_aggregate = (size_t)cap * 36 + fixed;
    p.lds_reduce = (size_t)p.bin_slots * 28;
    // bucket parts (one per XCD, fewer when fewer workgroups run): together
    // twice one record per vertex, each part a multiple of 4 records (whole
    // 128-byte lines)
    p.parts = p.ntiles < kXcds ? p.ntiles : kXcds;
    const uint64_t nparts = (uint64_t)p.nbins * p.parts;
    const uint64_t want = 2ull * (n ? n : 1);
    p.part_cap = (uint32_t)(((want + nparts - 1) / nparts + 3) / 4 * 4);
    p.off_cnt = 0;
    p.off_rec = align256(nparts * 4);
    p.bytes = p.off_rec + align256(nparts * p.part_cap * sizeof(Rec)) + 256;
    return p;
}

// Probe / claim like find_or_claim, without the occupancy bit (set by the
// reduce pass, which owns the bitmap words of its bin), from probe d0 at
// slot s onwards.
__device__ __forceinline__ uint32_t claim_next(const Tab &t, uint64_t key, uint32_t f, uint32_t s, uint32_t d0) {
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

__device__ __forceinline__ uint32_t claim(const Tab &t, uint64_t key) {
    return claim_next(t, key, fingerprint_of(key), home_of(key, t.mask), 0);
}

__device__ __forceinline__ void store_rec(Rec *p, uint32_t slot, uint32_t count, uint64_t s0, uint64_t s1,
                                          uint64_t s2) {
    uint4 *w = reinterpret_cast<uint4 *>(p);
    w[0] = make_uint4(slot, count, (uint32_t)s0, (uint32_t)(s0 >> 32));
    w[1] = make_uint4((uint32_t)s1, (uint32_t)(s1 >> 32), (uint32_t)s2, (uint32_t)(s2 >> 32));
}

// Key of vertex i built in the insert itself (Algorithm 1, as pf_build_keys);
// the caller has checked the vertex's valid byte.
__device__ __forceinline__ uint8_t fused_key(const FusedKeys &fk, uint32_t i, uint64_t &k) {
    const float x[3] = {fk.px[i], fk.py[i], fk.pz[i]};
    const float nr[3] = {fk.nx[i], fk.ny[i], fk.nz[i]};
    uint32_t fp, home;
    const PcgJump jp(fk.a.seed, fk.a.idx_base);
    return vertex_key(x, nr, true, fk.a.cam, fk.a.s, fk.a.inv_s, jp, i, fk.a.mask, k, fp, home);
}

// A group whose bucket part is full: its count and sums go to the cell by
// device atomics and its occupancy bit is set now (reduce sets the bits of
// the cells it receives records for).
__device__ __noinline__ void spill(const Tab &t, uint32_t s, uint32_t count, uint64_t s0, uint64_t s1, uint64_t s2) {
    accumulate(t, s, count, (int64_t)s0, (int64_t)s1, (int64_t)s2);
    __hip_atomic_fetch_or(&t.occ[s >> 5], 1u << (s & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Where the records of this workgroup's groups go: bin b's part `part` of
// `parts` (the workgroup's XCD), part_cap records each.
struct Buckets {
    uint32_t *cnt;
    Rec *rec;
    uint32_t bin_shift, parts, part, part_cap;
};

// Position of a record of slot s in its bin's bucket part.
__device__ __forceinline__ uint32_t bucket_pos(const Buckets &bk, uint32_t s) {
    return __hip_atomic_fetch_add(&bk.cnt[(s >> bk.bin_shift) * bk.parts + bk.part], 1u, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void put_rec(const Tab &t, const Buckets &bk, uint32_t pos, uint32_t s, uint32_t count,
                                        uint64_t s0, uint64_t s1, uint64_t s2) {
    if (pos < bk.part_cap)
        store_rec(bk.rec + ((size_t)(s >> bk.bin_shift) * bk.parts + bk.part) * bk.part_cap + pos, s, count, s0, s1,
                  s2);
    else
        spill(t, s, count, s0, s1, s2);
}

// kKeys: keys are built here from positions and normals (fk) and the flags
// are outputs only; otherwise key[] and flags[] come from pf_build_keys.
template <bool kKeys>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) void aggregate_kernel(
    Tab t, const uint64_t *__restrict__ key, const float *__restrict__ r, const float *__restrict__ g,
    const float *__restrict__ b, uint8_t *__restrict__ flags, uint32_t *__restrict__ slot_out, uint32_t n,
    uint32_t cap, Buckets bk, FusedKeys fk) {
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned long long *lkey = reinterpret_cast<unsigned long long *>(lds);
    unsigned long long *ls0 = lkey + cap, *ls1 = ls0 + cap, *ls2 = ls1 + cap;
    uint32_t *lcnt = reinterpret_cast<uint32_t *>(ls2 + cap);  // count, then the group's slot
    uint32_t *misc = lcnt + cap;                                // [0] listed vertices, [1] overflowed vertices
    uint16_t *vlist = reinterpret_cast<uint16_t *>(misc + 4);   // the chunk's valid vertices (local indices)
    uint16_t *vent = vlist + kChunk;                            // per local vertex: flags << 11 | entry
    if (threadIdx.x < 2) misc[threadIdx.x] = 0;
    bk.part = blockIdx.x % bk.parts;
    // chunks are dealt out with a stride so that every workgroup gets a mix
    // of coherent and incoherent (or empty) parts of the stream
    const uint32_t nchunks = (n + kChunk - 1) / kChunk;
    for (uint32_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {
        const uint32_t c0 = ci * kChunk;
        const uint32_t i1 = min(n, c0 + kChunk);
        if (threadIdx.x == 0) misc[0] = 0;
        for (uint32_t j = threadIdx.x; j < cap; j += kT) {
            lkey[j] = kEmpty;
            ls0[j] = 0;
            ls1[j] = 0;
            ls2[j] = 0;
            lcnt[j] = 0;
        }
        __syncthreads();
        // only the flags (8 bits per vertex) and the LDS entries (16 bits,
        // 0xffff = none) stay live across the barriers, packed; the rare
        // vertex that finds no room reloads its key and contribution
        uint32_t flp0 = 0, flp = 0;
        uint64_t ep = 0;
        uint32_t live = 0;
        if constexpr (kKeys) {
            flp0 = 0xffffffffu;  // no input flags: every vertex's flags are written
            // the valid bytes of the thread's vertices first: masked vertices
            // (sky, escaped paths) read nothing more.  The valid vertices are
            // listed (each wavefront's in one run, in vertex order), so that
            // key construction runs on full wavefronts: a bounce segment holds
            // about one valid vertex in four
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) {
                const uint32_t i = c0 + u * kT + threadIdx.x;
                const bool v = i < i1 && (fk.valid == nullptr || fk.valid[i] != 0);
                live |= (v ? 1u : 0u) << u;
            }
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) {
                const bool v = (live >> u) & 1u;
                const uint32_t pos = wave_reserve(&misc[0], v);
                if (v) vlist[pos] = (uint16_t)(u * kT + threadIdx.x);
            }
            __syncthreads();
            const uint32_t nlisted = misc[0];
#pragma unroll 1
            for (uint32_t j0 = 0; j0 < nlisted; j0 += kT) {
                const uint32_t j = j0 + threadIdx.x;
                const bool on = j < nlisted;
                const uint32_t li = on ? vlist[j] : 0u;
                const uint32_t i = c0 + li;
                uint32_t f = PF_V_INVALID;
                uint64_t k = 0;
                int64_t q0 = 0, q1 = 0, q2 = 0;
                if (on) {
                    const float cr = r[i], cg = g[i], cb = b[i];
                    f = fused_key(fk, i, k);
                    if (f == 0) f = fixed_point(cr, cg, cb, t.frac_bits, q0, q1, q2);
                    if (fk.key_out) fk.key_out[i] = k;
                }
                const int e = merge_into_lds<false>(lkey, ls0, ls1, ls2, lcnt, cap, on && f == 0, k, q0, q1, q2);
                if (on) vent[li] = (uint16_t)((f << 11) | (e < 0 ? 0x7ffu : (uint32_t)e));
            }
        } else {
#pragma unroll
        for (uint32_t u = 0; u < kPer; ++u) {
            const uint32_t i = c0 + u * kT + threadIdx.x;
            flp0 |= (uint32_t)(i < i1 ? flags[i] : (uint8_t)PF_V_INVALID) << (8 * u);
        }
        flp = flp0;
        // software pipeline: the contribution and key of vertex u + 1 are in
        // flight while vertex u is merged
        float nr = 0.0f, ng = 0.0f, nb = 0.0f;
        uint64_t nk = 0;
        if ((flp0 & 0xffu) == 0) {
            const uint32_t i = c0 + threadIdx.x;
            nr = r[i];
            ng = g[i];
            nb = b[i];
            nk = key[i];
        }
#pragma unroll 1
        for (uint32_t u = 0; u < kPer; ++u) {
            const float cr = nr, cg = ng, cb = nb;
            const uint64_t k = nk;
            if (u + 1 < kPer && ((flp0 >> (8 * (u + 1))) & 0xffu) == 0) {
                const uint32_t i = c0 + (u + 1) * kT + threadIdx.x;
                nr = r[i];
                ng = g[i];
                nb = b[i];
                nk = key[i];
            }
            uint32_t f = (flp0 >> (8 * u)) & 0xffu;
            int64_t q0 = 0, q1 = 0, q2 = 0;
            if (f == 0) f = fixed_point(cr, cg, cb, t.frac_bits, q0, q1, q2);
            flp |= f << (8 * u);  // bits change only where they were 0
            const int e = merge_into_lds<false>(lkey, ls0, ls1, ls2, lcnt, cap, f == 0, k, q0, q1, q2);
            ep |= (uint64_t)(uint16_t)e << (16 * u);
        }
        }
        __syncthreads();
        if constexpr (kKeys) {  // the thread's vertices' flags and entries, packed as in the other mode
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) {
                uint32_t f = PF_V_INVALID, e = 0xffffu;
                if ((live >> u) & 1u) {
                    const uint32_t ve = vent[u * kT + threadIdx.x];
                    f = ve >> 11;
                    e = (ve & 0x7ffu) == 0x7ffu ? 0xffffu : (ve & 0x7ffu);
                }
                flp |= f << (8 * u);
                ep |= (uint64_t)e << (16 * u);
            }
        }
        // one probe / claim and one record per group; a thread's entries
        // issue their home-slot loads, then their compare-and-swaps on empty
        // home slots, then their bucket positions, before any result is used
        uint64_t gk[kFlush];
        uint32_t fs[kFlush], ff[kFlush], fcur[kFlush];
#pragma unroll
        for (uint32_t v = 0; v < kFlush; ++v) {
            const uint32_t j = v * kT + threadIdx.x;
            gk[v] = j < cap ? lkey[j] : kEmpty;
            fs[v] = 0;
            ff[v] = 0;
            fcur[v] = 0;
            if (gk[v] != kEmpty) {
                fs[v] = home_of(gk[v], t.mask);
                ff[v] = fingerprint_of(gk[v]);
                fcur[v] = load_fp_probe(&t.cell_at(fs[v]).fp);
            }
        }
        bool won[kFlush];
#pragma unroll
        for (uint32_t v = 0; v < kFlush; ++v) {
            won[v] = false;
            if (gk[v] != kEmpty && fcur[v] == 0) {
                uint32_t expected = 0;
                won[v] = __hip_atomic_compare_exchange_strong(&t.cell_at(fs[v]).fp, &expected, ff[v], __ATOMIC_RELAXED,
                                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                fcur[v] = won[v] ? ff[v] : expected;
            }
        }
        uint32_t sl[kFlush], pos[kFlush];
#pragma unroll
        for (uint32_t v = 0; v < kFlush; ++v) {
            const uint32_t j = v * kT + threadIdx.x;
            sl[v] = kNoSlot;
            pos[v] = 0;
            if (gk[v] != kEmpty) {
                if (won[v]) t.key_at(fs[v]) = gk[v];
                // the home slot holds another key: probe on from the next
                sl[v] = fcur[v] == ff[v] ? fs[v] : claim_next(t, gk[v], ff[v], (fs[v] + 1) & t.mask, 1);
                if (sl[v] == kNoSlot)
                    atomicAdd(&misc[1], lcnt[j]);
                else
                    pos[v] = bucket_pos(bk, sl[v]);
            }
        }
#pragma unroll
        for (uint32_t v = 0; v < kFlush; ++v) {
            const uint32_t j = v * kT + threadIdx.x;
            if (gk[v] != kEmpty) {
                if (sl[v] != kNoSlot)
                    put_rec(t, bk, pos[v], sl[v], lcnt[j], ls0[j], ls1[j], ls2[j]);
                lcnt[j] = sl[v];
            }
        }
        __syncthreads();
#pragma unroll 1
        for (uint32_t u = 0; u < kPer; ++u) {
            const uint32_t i = c0 + u * kT + threadIdx.x;
            uint32_t f = (flp >> (8 * u)) & 0xffu;
            const uint32_t e = (uint32_t)(ep >> (16 * u)) & 0xffffu;
            uint32_t s = kNoSlot;
            if (f == 0) {
                if (e != 0xffffu) {
                    s = lcnt[e];
                } else {  // no room in the LDS table: a group of its own
                    int64_t q0, q1, q2;
                    fixed_point(r[i], g[i], b[i], t.frac_bits, q0, q1, q2);
                    uint64_t k;
                    if constexpr (kKeys)
                        fused_key(fk, i, k);
                    else
                        k = key[i];
                    s = claim(t, k);
                    if (s != kNoSlot)
                        put_rec(t, bk, bucket_pos(bk, s), s, 1u, (uint64_t)q0, (uint64_t)q1, (uint64_t)q2);
                    else
                        atomicAdd(&misc[1], 1u);
                }
                if (s == kNoSlot) f = PF_V_OVERFLOW;
            }
            if (i < i1) {
                if (f != ((flp0 >> (8 * u)) & 0xffu)) flags[i] = (uint8_t)f;
                slot_out[i] = s;
                if constexpr (kKeys)
                    if (fk.key_out && !((live >> u) & 1u)) fk.key_out[i] = 0;
            }
        }
        __syncthreads();  // the table is cleared for the next chunk
    }
    if (threadIdx.x == 0 && misc[1]) add_u64(&t.stats[PF_STAT_PART_OVF + (blockIdx.x & 15)], misc[1]);
}

__global__ void zero_kernel(uint32_t *__restrict__ p, uint32_t m) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) p[j] = 0;
}

constexpr uint32_t kBatch = 4;  // records per thread loaded before any is used

// The temporal blend done by reduce: the previous table (has_prev) and the
// blend's parameters as pf_temporal_update / pf_temporal_integrate take them.
struct Blend {
    Tab prev;
    float alpha, beta;
    uint32_t cap;
};

// One workgroup per bin: LDS sums over its records (the bucket parts of
// the XCDs), then the exclusive owner adds them to the cells and sets the
// occupancy bits of its words.  kBlend: the owner then computes the temporal
// values of its cells (the cells are final: every record of a slot is in the
// slot's bin, and spilled groups went to their cells before this launch), as
// temporal_word does for one bitmap word.
template <bool kBlend = false, bool kHasPrev = false, bool kIntegrate = false>
__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(Tab t, const Rec *__restrict__ rec,
                                                                const uint32_t *__restrict__ cnt_parts,
                                                                uint32_t parts, uint32_t part_cap, uint32_t bin_slots,
                                                                Blend bl) {
    extern __shared__ unsigned long long lred[];
    unsigned long long *sum0 = lred, *sum1 = lred + bin_slots, *sum2 = lred + 2 * bin_slots;
    uint32_t *cnt = reinterpret_cast<uint32_t *>(lred + 3 * bin_slots);
    __shared__ uint32_t seg[kXcds + 1];    // running record counts of the parts
    __shared__ uint32_t spilled[4096 / 32];  // occupancy bits set by spilled groups (kBlend)
    const uint32_t bin = blockIdx.x;
    const uint32_t base = bin * bin_slots;
    for (uint32_t k = threadIdx.x; k < bin_slots; k += kReduceThreads) {
        sum0[k] = 0;
        sum1[k] = 0;
        sum2[k] = 0;
        cnt[k] = 0;
    }
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t x = 0; x < kXcds; ++x) {
            seg[x] = acc;
            const uint32_t c = x < parts ? cnt_parts[bin * parts + x] : 0u;
            acc += c < part_cap ? c : part_cap;
        }
        seg[kXcds] = acc;
    }
    if constexpr (kBlend) {
        // before this launch only spilled groups set bits (the table was
        // empty before the insert)
        for (uint32_t w = threadIdx.x; w < (bin_slots + 31) / 32; w += kReduceThreads)
            spilled[w] = t.occ[(base >> 5) + w];
    }
    __syncthreads();
    const uint4 *in = reinterpret_cast<const uint4 *>(rec + (size_t)bin * parts * part_cap);
    const uint32_t j1 = seg[kXcds];
    for (uint32_t jb = 0; jb < j1; jb += kBatch * kReduceThreads) {
        uint4 lo[kBatch], hi[kBatch];
#pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) {
            const uint32_t j = jb + u * kReduceThreads + threadIdx.x;
            if (j < j1) {
                uint32_t x = 0;
#pragma unroll
                for (uint32_t y = 1; y < kXcds; ++y) x = j >= seg[y] ? y : x;
                const size_t at = (size_t)x * part_cap + (j - seg[x]);
                lo[u] = in[2 * at];
                hi[u] = in[2 * at + 1];
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) {
            const uint32_t j = jb + u * kReduceThreads + threadIdx.x;
            if (j < j1) {
                const uint32_t loc = lo[u].x - base;
                atomicAdd(&cnt[loc], lo[u].y);
                atomicAdd(&sum0[loc], (unsigned long long)lo[u].z | (unsigned long long)lo[u].w << 32);
                atomicAdd(&sum1[loc], (unsigned long long)hi[u].x | (unsigned long long)hi[u].y << 32);
                atomicAdd(&sum2[loc], (unsigned long long)hi[u].z | (unsigned long long)hi[u].w << 32);
            }
        }
    }
    __syncthreads();
    // the cells of a thread's slots are all loaded before any is updated
    uint4 *cells = t.words_at(base);  // 4 sixteen-byte words per slot record
    uint32_t hits = 0;
    for (uint32_t kb = 0; kb < bin_slots; kb += kBatch * kReduceThreads) {
        uint32_t c[kBatch];
        uint4 lo[kBatch], hi[kBatch];
#pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) {
            const uint32_t k = kb + u * kReduceThreads + threadIdx.x;
            c[u] = k < bin_slots ? cnt[k] : 0u;
            if (c[u]) {
                lo[u] = cells[4 * k];
                hi[u] = cells[4 * k + 1];
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) {
            const uint32_t k = kb + u * kReduceThreads + threadIdx.x;
            if (c[u]) {
                const uint64_t s0 = ((uint64_t)lo[u].z | (uint64_t)lo[u].w << 32) + sum0[k];
                const uint64_t s1 = ((uint64_t)hi[u].x | (uint64_t)hi[u].y << 32) + sum1[k];
                const uint64_t s2 = ((uint64_t)hi[u].z | (uint64_t)hi[u].w << 32) + sum2[k];
                cells[4 * k] = make_uint4(lo[u].x, lo[u].y + c[u], (uint32_t)s0, (uint32_t)(s0 >> 32));
                cells[4 * k + 1] = make_uint4((uint32_t)s1, (uint32_t)(s1 >> 32), (uint32_t)s2, (uint32_t)(s2 >> 32));
            }
            // occupancy: a wavefront's 64 consecutive slots are two bitmap
            // words of this bin (bins hold >= 32 slots, or the whole table)
            const uint64_t m = __ballot(c[u] != 0);
            if ((threadIdx.x & 63) == 0 && m) {
                const uint32_t w = (base + k) >> 5;
                if ((uint32_t)m) t.occ[w] |= (uint32_t)m;
                if (m >> 32) t.occ[w + 1] |= (uint32_t)(m >> 32);
            }
        }
    }
    if constexpr (kBlend) {
        // the bin's cells are final: listed in LDS (the sums' space is free
        // now), then blended one per lane, so that every lane has a cell
        // while the list lasts
        __shared__ uint32_t nlist, s_hits;
        uint32_t *list = reinterpret_cast<uint32_t *>(sum0);
        if (threadIdx.x == 0) {
            nlist = 0;
            s_hits = 0;
        }
        __syncthreads();  // the cells are written, the sums no longer read
        for (uint32_t k = threadIdx.x; k < bin_slots; k += kReduceThreads)
            if (cnt[k] || ((spilled[k >> 5] >> (k & 31)) & 1u)) list[atomicAdd(&nlist, 1u)] = k;
        __syncthreads();
        const uint32_t m = nlist;
        for (uint32_t q = threadIdx.x; q < m; q += kReduceThreads) {
            const uint32_t sl[1] = {base + list[q]};
            const uint4 *w4 = t.words_at(sl[0]);  // written above by this workgroup
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
            uint32_t keep[1] = {kIntegrate ? min(cl.count, bl.cap) : cl.count};
            float v[1][3] = {{t.average(cl, 0), t.average(cl, 1), t.average(cl, 2)}};
            hits += blend_cells<kHasPrev, kIntegrate, 1, false>(t, bl.prev, sl, has, key, fp, v, n, keep, bl.alpha,
                                                                bl.beta, bl.cap);
        }
        if constexpr (kHasPrev) {
            // one device atomic per workgroup, spread over 32 partial counters
            if (hits) atomicAdd(&s_hits, hits);
            __syncthreads();
            if (threadIdx.x == 0 && s_hits) add_u64(&t.stats[PF_STAT_PART_HIT + (blockIdx.x & 31)], s_hits);
        }
    }
}

}  // namespace binned

size_t binned_workspace_bytes(uint32_t n, uint32_t log2_slots) {
    if (log2_slots > binned::kMaxLog2Slots) return 0;
    return binned::make_plan(n, log2_slots).bytes;
}

namespace binned {

// the reduce kernels of every blend variant, for their LDS attribute
static const void *const kReduceKernels[] = {
    reinterpret_cast<const void *>(reduce_kernel<false, false, false>),
    reinterpret_cast<const void *>(reduce_kernel<true, false, false>),
    reinterpret_cast<const void *>(reduce_kernel<true, true, false>),
    reinterpret_cast<const void *>(reduce_kernel<true, false, true>),
    reinterpret_cast<const void *>(reduce_kernel<true, true, true>)};

// blend: NULL for the insert alone; else the temporal blend in reduce
// (has_prev: blend->prev is a table; integrate: temporal integration).
template <bool kKeys>
static hipError_t run(const Tab &t, const uint64_t *key, const float *r, const float *g, const float *b,
                      uint8_t *flags, uint32_t *slot_out, uint32_t n, void *ws, const FusedKeys &fk,
                      const Blend *blend, bool has_prev, bool integrate, hipStream_t st) {
    const uint32_t log2_slots = 32 - __builtin_clz(t.mask + 1) - 1;
    const Plan p = make_plan(n, log2_slots);
    char *base = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(ws) + 255) / 256 * 256);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(base + p.off_cnt);
    Rec *rec = reinterpret_cast<Rec *>(base + p.off_rec);
    static bool attrs = false;  // dynamic LDS above 64 KB needs the attribute, set once per function
    if (!attrs) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(aggregate_kernel<false>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(aggregate_kernel<true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget);
        for (const void *f : kReduceKernels)
            if (e == hipSuccess)
                e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(4096 * 28));
        if (e != hipSuccess) return e;
        attrs = true;
    }
    const uint32_t nparts = p.nbins * p.parts;
    zero_kernel<<<(nparts + 1023) / 1024 < 256 ? (nparts + 1023) / 1024 : 256, 1024, 0, st>>>(cnt, nparts);
    const Buckets bk{cnt, rec, p.bin_shift, p.parts, 0, p.part_cap};
    aggregate_kernel<kKeys><<<p.ntiles, kT, p.lds_aggregate, st>>>(t, key, r, g, b, flags, slot_out, n, p.cap, bk,
                                                                   fk);
    const Blend none{};
    const Blend &bl = blend ? *blend : none;
    if (!blend)
        reduce_kernel<<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, cnt, p.parts, p.part_cap, p.bin_slots, bl);
    else if (!has_prev && !integrate)
        reduce_kernel<true, false, false><<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, cnt, p.parts, p.part_cap,
                                                                                       p.bin_slots, bl);
    else if (has_prev && !integrate)
        reduce_kernel<true, true, false><<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, cnt, p.parts, p.part_cap,
                                                                                      p.bin_slots, bl);
    else if (!has_prev)
        reduce_kernel<true, false, true><<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, cnt, p.parts, p.part_cap,
                                                                                      p.bin_slots, bl);
    else
        reduce_kernel<true, true, true><<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, cnt, p.parts, p.part_cap,
                                                                                     p.bin_slots, bl);
    return hipGetLastError();
}

}  // namespace binned

hipError_t launch_insert_binned(const Tab &t, const uint64_t *key, const float *r, const float *g, const float *b,
                                uint8_t *flags, uint32_t *slot_out, uint32_t n, void *ws, hipStream_t st) {
    binned::FusedKeys none{};
    return binned::run<false>(t, key, r, g, b, flags, slot_out, n, ws, none, nullptr, false, false, st);
}

hipError_t launch_keys_insert_binned(const Tab &t, const float *px, const float *py, const float *pz,
                                     const float *nx, const float *ny, const float *nz, const uint8_t *valid,
                                     const KeyArgs &a, uint64_t *key_out, const float *r, const float *g,
                                     const float *b, uint8_t *flags, uint32_t *slot_out, uint32_t n, void *ws,
                                     hipStream_t st) {
    const binned::FusedKeys fk{px, py, pz, nx, ny, nz, valid, a, key_out};
    return binned::run<true>(t, nullptr, r, g, b, flags, slot_out, n, ws, fk, nullptr, false, false, st);
}

hipError_t launch_keys_insert_binned_temporal(const Tab &t, const float *px, const float *py, const float *pz,
                                              const float *nx, const float *ny, const float *nz,
                                              const uint8_t *valid, const KeyArgs &a, uint64_t *key_out,
                                              const float *r, const float *g, const float *b, uint8_t *flags,
                                              uint32_t *slot_out, uint32_t n, void *ws, const Tab *prev,
                                              float alpha_old, int mode, uint32_t cap, hipStream_t st) {
    const binned::FusedKeys fk{px, py, pz, nx, ny, nz, valid, a, key_out};
    binned::Blend bl{};
    if (prev) bl.prev = *prev;
    bl.alpha = alpha_old;
    bl.beta = 1.0f - alpha_old;
    bl.cap = cap;
    return binned::run<true>(t, nullptr, r, g, b, flags, slot_out, n, ws, fk, &bl, prev != nullptr, mode == 1, st);
}

// ---- the insert without a workspace argument, for callers that cannot
// allocate.  Its workspace is a file-scope device array; on the host the
// array's name is not a device address, so every use goes through the
// address hipGetSymbolAddress returns for the current device (kept per
// device).  All calls on one device share the array: calls that overlap in
// time on one device (different streams, or host threads) race.

namespace binned {

constexpr uint32_t kNoAllocBatch = PF_NOALLOC_BATCH;  // vertices per pass over the scratch
constexpr size_t kScratchBytes = PF_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex scratch_mutex;
static void *scratch_ptr[kMaxDevices];

// The current device's address of `scratch`, looked up once per device.
static hipError_t scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace binned

bool noalloc_fits(uint32_t log2_slots) {
    return log2_slots <= binned::kMaxLog2Slots &&
           binned::make_plan(binned::kNoAllocBatch, log2_slots).bytes + 256 <= binned::kScratchBytes;
}

hipError_t launch_keys_insert_binned_noalloc(const Tab &t, const float *px, const float *py, const float *pz,
                                             const float *nx, const float *ny, const float *nz,
                                             const uint8_t *valid, const KeyArgs &a, uint64_t *key_out,
                                             const float *r, const float *g, const float *b, uint8_t *flags,
                                             uint32_t *slot_out, uint32_t n, hipStream_t st) {
    void *ws = nullptr;
    hipError_t e = binned::scratch_address(&ws);
    if (e != hipSuccess) return e;
    // the insert accumulates, so consecutive batches give the table one
    // call would; each batch's workspace is written before it is read
    for (uint32_t i0 = 0; i0 < n; i0 += binned::kNoAllocBatch) {
        const uint32_t m = n - i0 < binned::kNoAllocBatch ? n - i0 : binned::kNoAllocBatch;
        const uint32_t log2_slots = 32 - __builtin_clz(t.mask + 1) - 1;
        if (binned::make_plan(m, log2_slots).bytes + 256 > binned::kScratchBytes) return hipErrorInvalidValue;
        KeyArgs ab = a;
        ab.idx_base = a.idx_base + i0;
        const binned::FusedKeys fk{px + i0, py + i0, pz + i0, nx + i0, ny + i0, nz + i0,
                                   valid ? valid + i0 : nullptr, ab, key_out ? key_out + i0 : nullptr};
        e = binned::run<true>(t, nullptr, r + i0, g + i0, b + i0, flags + i0, slot_out + i0, m, ws, fk, nullptr,
                              false, false, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace pfk
