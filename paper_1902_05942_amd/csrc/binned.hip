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
//              kernel); each group then probes / claims its cell
//              once (compare-and-swap on new cells only), writes one record
//              {slot, count, sums} to the tile's staging area and counts it
//              in the tile's histogram of slot bins; every vertex receives
//              its group's slot
//   colscan    per bin: running record offsets over the tiles, bin totals
//   scatter    per tile: the start offset of every bin (each workgroup scans
//              the bin totals itself), then staged records moved to their
//              bin's range
//   reduce     per bin (a contiguous slot range): records summed in LDS, then
//              count and sums added to the cells with plain loads and stores
//              by the workgroup that owns them, occupancy bits set; with a
//              temporal blend (Section 3.4.1) in the same launch, the owner
//              also blends each cell's final average with the previous
//              table's value of its key and stores the temporal value
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

struct Plan {
    uint32_t log2_bins, nbins, bin_shift, bin_slots, ntiles, tile, cap;
    size_t lds_aggregate, lds_reduce;
    size_t off_h, off_tot, off_start, off_ntr, off_trec, off_rec, bytes;
};

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

Plan make_plan(uint32_t n, uint32_t log2_slots) {
    Plan p;
    // bins of 2048 slots (4096 above 2^24 slots, keeping the histogram small)
    uint32_t lbs = log2_slots > 24 ? 12 : 11;
    if (lbs > log2_slots) lbs = log2_slots;
    p.bin_shift = lbs;
    p.bin_slots = 1u << lbs;
    p.log2_bins = log2_slots - lbs;
    p.nbins = 1u << p.log2_bins;
    // a tile is the set of chunks one workgroup takes (every ntiles-th);
    // its staging area holds a record per vertex at most
    const uint32_t nchunks = (n + kChunk - 1) / kChunk;
    p.ntiles = nchunks < kMaxTiles ? (nchunks ? nchunks : 1) : kMaxTiles;
    p.tile = (nchunks + p.ntiles - 1) / p.ntiles * kChunk;
    if (p.tile == 0) p.tile = kChunk;
    // LDS of aggregate: key 8 B, sums 24 B and count 4 B per entry, the bin
    // histogram and two counters; entries take what the budget leaves
    const size_t fixed = (size_t)p.nbins * 4 + 16;
    uint32_t cap = (uint32_t)((kLdsBudget - fixed) / 36) / 64 * 64;
    if (cap < 512) cap = 512;
    if (cap > kFlush * kT) cap = kFlush * kT;
    p.cap = cap;
    p.lds_aggregate = (size_t)cap * 36 + fixed;
    p.lds_reduce = (size_t)p.bin_slots * 28;
    p.off_h = 0;
    p.off_tot = align256((size_t)p.ntiles * p.nbins * 4);
    p.off_start = p.off_tot + align256((size_t)p.nbins * 4);
    p.off_ntr = p.off_start + align256((size_t)p.nbins * 4);
    p.off_trec = p.off_ntr + align256((size_t)p.ntiles * 4);
    p.off_rec = p.off_trec + align256((size_t)p.ntiles * p.tile * sizeof(Rec));
    p.bytes = p.off_rec + align256((size_t)(n ? n : 1) * sizeof(Rec)) + 256;
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

// kKeys: keys are built here from positions and normals (fk) and the flags
// are outputs only; otherwise key[] and flags[] come from pf_build_keys.
template <bool kKeys>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) void aggregate_kernel(
    Tab t, const uint64_t *__restrict__ key, const float *__restrict__ r, const float *__restrict__ g,
    const float *__restrict__ b, uint8_t *__restrict__ flags, uint32_t *__restrict__ slot_out, uint32_t n,
    uint32_t tile, uint32_t cap, uint32_t nbins, uint32_t bin_shift, uint32_t *__restrict__ H,
    uint32_t *__restrict__ ntr, Rec *__restrict__ trec, FusedKeys fk) {
    extern __shared__ __align__(16) unsigned char lds[];
    unsigned long long *lkey = reinterpret_cast<unsigned long long *>(lds);
    unsigned long long *ls0 = lkey + cap, *ls1 = ls0 + cap, *ls2 = ls1 + cap;
    uint32_t *lcnt = reinterpret_cast<uint32_t *>(ls2 + cap);  // count, then the group's slot
    uint32_t *hist = lcnt + cap;
    uint32_t *misc = hist + nbins;                              // [0] staged records, [1] overflowed vertices
    for (uint32_t k = threadIdx.x; k < nbins; k += kT) hist[k] = 0;
    if (threadIdx.x < 2) misc[threadIdx.x] = 0;
    // chunks are dealt out with a stride so that every workgroup gets a mix
    // of coherent and incoherent (or empty) parts of the stream
    const uint32_t nchunks = (n + kChunk - 1) / kChunk;
    Rec *out = trec + (size_t)blockIdx.x * tile;
    for (uint32_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {
        const uint32_t c0 = ci * kChunk;
        const uint32_t i1 = min(n, c0 + kChunk);
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
        if constexpr (kKeys) {
            flp0 = 0xffffffffu;  // no input flags: every vertex's flags are written
            // the valid bytes of the thread's vertices first: masked vertices
            // (sky, escaped paths) read nothing more
            uint32_t live = 0;
#pragma unroll
            for (uint32_t u = 0; u < kPer; ++u) {
                const uint32_t i = c0 + u * kT + threadIdx.x;
                const bool v = i < i1 && (fk.valid == nullptr || fk.valid[i] != 0);
                live |= (v ? 1u : 0u) << u;
            }
#pragma unroll 1
            for (uint32_t u = 0; u < kPer; ++u) {
                const uint32_t i = c0 + u * kT + threadIdx.x;
                uint32_t f = PF_V_INVALID;
                uint64_t k = 0;
                int64_t q0 = 0, q1 = 0, q2 = 0;
                if ((live >> u) & 1u) {
                    const float cr = r[i], cg = g[i], cb = b[i];
                    f = fused_key(fk, i, k);
                    if (f == 0) f = fixed_point(cr, cg, cb, t.frac_bits, q0, q1, q2);
                }
                if (fk.key_out && i < i1) fk.key_out[i] = k;
                flp |= f << (8 * u);
                const int e = merge_into_lds<false>(lkey, ls0, ls1, ls2, lcnt, cap, f == 0, k, q0, q1, q2);
                ep |= (uint64_t)(uint16_t)e << (16 * u);
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
        // one probe / claim and one staged record per group; a thread's
        // entries issue their home-slot loads, then their compare-and-swaps
        // on empty home slots, before either result is needed
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
#pragma unroll
        for (uint32_t v = 0; v < kFlush; ++v) {
            const uint32_t j = v * kT + threadIdx.x;
            uint32_t s = kNoSlot;
            if (gk[v] != kEmpty) {
                if (won[v]) t.key_at(fs[v]) = gk[v];
                // the home slot holds another key: probe on from the next
                s = fcur[v] == ff[v] ? fs[v] : claim_next(t, gk[v], ff[v], (fs[v] + 1) & t.mask, 1);
                if (s == kNoSlot) atomicAdd(&misc[1], lcnt[j]);
            }
            const bool stage = gk[v] != kEmpty && s != kNoSlot;
            const uint32_t pos = wave_reserve(&misc[0], stage);
            if (stage) {
                store_rec(out + pos, s, lcnt[j], ls0[j], ls1[j], ls2[j]);
                atomicAdd(&hist[s >> bin_shift], 1u);
            }
            if (gk[v] != kEmpty) lcnt[j] = s;
        }
        __syncthreads();
#pragma unroll 1
        for (uint32_t u = 0; u < kPer; ++u) {
            const uint32_t i = c0 + u * kT + threadIdx.x;
            uint32_t f = (flp >> (8 * u)) & 0xffu;
            const uint32_t e = (uint32_t)(ep >> (16 * u)) & 0xffffu;
            uint32_t s = kNoSlot;
            bool alone = false;
            int64_t q0 = 0, q1 = 0, q2 = 0;
            if (f == 0) {
                if (e != 0xffffu) {
                    s = lcnt[e];
                } else {  // no room in the LDS table: a group of its own
                    fixed_point(r[i], g[i], b[i], t.frac_bits, q0, q1, q2);
                    uint64_t k;
                    if constexpr (kKeys)
                        fused_key(fk, i, k);
                    else
                        k = key[i];
                    s = claim(t, k);
                    alone = s != kNoSlot;
                    if (!alone) atomicAdd(&misc[1], 1u);
                }
                if (s == kNoSlot) f = PF_V_OVERFLOW;
            }
            const uint32_t pos = wave_reserve(&misc[0], alone);
            if (alone) {
                store_rec(out + pos, s, 1u, (uint64_t)q0, (uint64_t)q1, (uint64_t)q2);
                atomicAdd(&hist[s >> bin_shift], 1u);
            }
            if (i < i1) {
                if (f != ((flp0 >> (8 * u)) & 0xffu)) flags[i] = (uint8_t)f;
                slot_out[i] = s;
            }
        }
        __syncthreads();  // the table is cleared for the next chunk
    }
    __syncthreads();
    uint32_t *row = H + (size_t)blockIdx.x * nbins;
    for (uint32_t k = threadIdx.x; k < nbins; k += kT) row[k] = hist[k];
    if (threadIdx.x == 0) {
        ntr[blockIdx.x] = misc[0];
        if (misc[1]) add_u64(&t.stats[PF_STAT_PART_OVF + (blockIdx.x & 15)], misc[1]);
    }
}

// Per bin: exclusive running offset over the tiles (in place), bin total.
// Tiles are taken XCD by XCD (workgroups are dealt to the 8 XCDs in turn,
// so tile t runs on XCD t % 8): a bin's range is cut into 8 sub-ranges each
// written by the scatter workgroups of one XCD, and a cache line of records
// is filled through one L2 instead of several.
// A workgroup takes 16 bins; each of its 64 rows of lanes holds the counts of
// 8 consecutive tiles of that order in registers, so a column is loaded
// once, summed in parallel and rewritten without a second read.
constexpr int kScanBins = 16, kScanRows = 64, kScanPer = 8;
constexpr uint32_t kXcds = 8;
static_assert(kScanRows * kScanPer >= kMaxTiles, "one register batch covers every tile");
static_assert(kMaxTiles % kXcds == 0, "tiles split evenly over the XCDs");
__global__ __launch_bounds__(kScanBins *kScanRows) void colscan_kernel(uint32_t *__restrict__ H, uint32_t ntiles,
                                                                       uint32_t nbins,
                                                                       uint32_t *__restrict__ total) {
    __shared__ uint32_t part[kScanRows][kScanBins + 1];
    const uint32_t bx = threadIdx.x % kScanBins, cy = threadIdx.x / kScanBins;
    const uint32_t bin = blockIdx.x * kScanBins + bx;
    const uint32_t per = (ntiles + kXcds - 1) / kXcds;  // tiles per XCD (at most 64)
    const uint32_t q0 = cy * kScanPer;
    uint32_t v[kScanPer], tt[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const uint32_t q = q0 + k;  // position in XCD-major order
        tt[k] = (q % per) * kXcds + q / per;
        const bool in = bin < nbins && q < kXcds * per && tt[k] < ntiles;
        if (!in) tt[k] = ~0u;
        v[k] = in ? H[(size_t)tt[k] * nbins + bin] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s += v[k];
    part[cy][bx] = s;
    __syncthreads();
    uint32_t run = 0;
    for (uint32_t c = 0; c < cy; ++c) run += part[c][bx];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (tt[k] != ~0u) H[(size_t)tt[k] * nbins + bin] = run;
        run += v[k];
    }
    if (cy == kScanRows - 1 && bin < nbins) total[bin] = run;
}

constexpr uint32_t kBatch = 4;  // records per thread loaded before any is moved

__global__ __launch_bounds__(kT) void scatter_kernel(const Rec *__restrict__ trec, const uint32_t *__restrict__ ntr,
                                                     uint32_t tile, uint32_t nbins, uint32_t bin_shift,
                                                     const uint32_t *__restrict__ H,
                                                     const uint32_t *__restrict__ total, uint32_t *__restrict__ start,
                                                     Rec *__restrict__ rec) {
    extern __shared__ uint32_t cursor[];
    __shared__ uint32_t part[kT];
    const uint4 *in = reinterpret_cast<const uint4 *>(trec + (size_t)blockIdx.x * tile);
    const uint32_t m = ntr[blockIdx.x];
    uint4 lo[kBatch], hi[kBatch];
#pragma unroll
    for (uint32_t u = 0; u < kBatch; ++u) {  // first batch in flight while the cursors are set up
        const uint32_t j = u * kT + threadIdx.x;
        if (j < m) {
            lo[u] = in[2 * j];
            hi[u] = in[2 * j + 1];
        }
    }
    // every workgroup scans the bin totals itself (a few KB, L2-resident)
    // instead of waiting for a launch of its own; workgroup 0 stores the
    // bins' start offsets for reduce.  Each lane takes `per` consecutive
    // bins; a Hillis-Steele scan runs over the lanes' partial sums.
    const uint32_t *row = H + (size_t)blockIdx.x * nbins;
    const uint32_t per = (nbins + kT - 1) / kT;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t local = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < nbins) local += total[b0 + k];
    part[threadIdx.x] = local;
    __syncthreads();
    for (uint32_t off = 1; off < kT; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - local;  // exclusive
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < nbins) {
            cursor[b0 + k] = run + row[b0 + k];
            if (blockIdx.x == 0) start[b0 + k] = run;
            run += total[b0 + k];
        }
    __syncthreads();
    for (uint32_t j0 = 0; j0 < m; j0 += kBatch * kT) {
        if (j0) {
#pragma unroll
            for (uint32_t u = 0; u < kBatch; ++u) {
                const uint32_t j = j0 + u * kT + threadIdx.x;
                if (j < m) {
                    lo[u] = in[2 * j];
                    hi[u] = in[2 * j + 1];
                }
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) {
            const uint32_t j = j0 + u * kT + threadIdx.x;
            if (j < m) {
                const uint32_t pos = atomicAdd(&cursor[lo[u].x >> bin_shift], 1u);
                uint4 *o = reinterpret_cast<uint4 *>(rec + pos);
                o[0] = lo[u];
                o[1] = hi[u];
            }
        }
    }
}

// The temporal blend done by reduce: the previous table (has_prev) and the
// blend's parameters as pf_temporal_update / pf_temporal_integrate take them.
struct Blend {
    Tab prev;
    float alpha, beta;
    uint32_t cap;
};

// One workgroup per bin: LDS sums over its records, then the exclusive
// owner adds them to the cells and sets the occupancy bits of its words.
// kBlend: the owner then computes the temporal values of its cells (the
// cells are final: every record of a slot is in the slot's bin), as
// temporal_word does for one bitmap word.
template <bool kBlend = false, bool kHasPrev = false, bool kIntegrate = false>
__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(Tab t, const Rec *__restrict__ rec,
                                                                const uint32_t *__restrict__ start,
                                                                const uint32_t *__restrict__ total,
                                                                uint32_t bin_slots, Blend bl) {
    extern __shared__ unsigned long long lred[];
    unsigned long long *sum0 = lred, *sum1 = lred + bin_slots, *sum2 = lred + 2 * bin_slots;
    uint32_t *cnt = reinterpret_cast<uint32_t *>(lred + 3 * bin_slots);
    const uint32_t bin = blockIdx.x;
    const uint32_t base = bin * bin_slots;
    for (uint32_t k = threadIdx.x; k < bin_slots; k += kReduceThreads) {
        sum0[k] = 0;
        sum1[k] = 0;
        sum2[k] = 0;
        cnt[k] = 0;
    }
    __syncthreads();
    const uint4 *in = reinterpret_cast<const uint4 *>(rec);
    const uint32_t j0 = start[bin], j1 = j0 + total[bin];
    for (uint32_t jb = j0; jb < j1; jb += kBatch * kReduceThreads) {
        uint4 lo[kBatch], hi[kBatch];
#pragma unroll
        for (uint32_t u = 0; u < kBatch; ++u) {
            const uint32_t j = jb + u * kReduceThreads + threadIdx.x;
            if (j < j1) {
                lo[u] = in[2 * (size_t)j];
                hi[u] = in[2 * (size_t)j + 1];
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
            if (cnt[k]) list[atomicAdd(&nlist, 1u)] = k;
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
    uint32_t *H = reinterpret_cast<uint32_t *>(base + p.off_h);
    uint32_t *tot = reinterpret_cast<uint32_t *>(base + p.off_tot);
    uint32_t *start = reinterpret_cast<uint32_t *>(base + p.off_start);
    uint32_t *ntr = reinterpret_cast<uint32_t *>(base + p.off_ntr);
    Rec *trec = reinterpret_cast<Rec *>(base + p.off_trec);
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
    aggregate_kernel<kKeys><<<p.ntiles, kT, p.lds_aggregate, st>>>(t, key, r, g, b, flags, slot_out, n, p.tile, p.cap,
                                                                   p.nbins, p.bin_shift, H, ntr, trec, fk);
    colscan_kernel<<<(p.nbins + kScanBins - 1) / kScanBins, kScanBins * kScanRows, 0, st>>>(H, p.ntiles, p.nbins,
                                                                                          tot);
    scatter_kernel<<<p.ntiles, kT, (size_t)p.nbins * 4, st>>>(trec, ntr, p.tile, p.nbins, p.bin_shift, H, tot,
                                                              start, rec);
    const Blend none{};
    const Blend &bl = blend ? *blend : none;
    if (!blend)
        reduce_kernel<<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, start, tot, p.bin_slots, bl);
    else if (!has_prev && !integrate)
        reduce_kernel<true, false, false><<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, start, tot,
                                                                                       p.bin_slots, bl);
    else if (has_prev && !integrate)
        reduce_kernel<true, true, false><<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, start, tot,
                                                                                      p.bin_slots, bl);
    else if (!has_prev)
        reduce_kernel<true, false, true><<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, start, tot,
                                                                                      p.bin_slots, bl);
    else
        reduce_kernel<true, true, true><<<p.nbins, kReduceThreads, p.lds_reduce, st>>>(t, rec, start, tot,
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
