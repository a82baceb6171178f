// Insert-accumulate without device atomics on the cells, for gfx950.
//
// Device atomics run at ~24 G/s on MI355X whatever the footprint, so the
// per-vertex atomic adds of the cell update bound the atomic insert.  Here
// the vertices are binned by the slot they were given and every bin (a
// contiguous slot range) is reduced by one workgroup in LDS, which then owns
// its cells and updates them with plain loads and stores:
//   claim    per vertex: fixed point, probe / claim (CAS on new cells only),
//            slot out, and a per-tile histogram of bins in LDS
//   colscan  per bin: running offsets over the tiles, bin totals
//   binscan  bin start offsets (one workgroup)
//   scatter  per vertex: record {slot, r, g, b} into its bin's range
//   reduce   per bin: LDS sums over the bin's records, then count and sums
//            added to the cells and the occupancy bits set (exclusive owner)
// Integer sums make the result identical to the atomic insert.
#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

namespace binned {

constexpr int kT = 1024;                 // threads of the tile kernels
constexpr uint32_t kLog2MinBinSlots = 10;
constexpr uint32_t kLog2MaxBins = 13;    // LDS histogram of 8192 bins
constexpr uint32_t kMaxLog2Slots = 25;   // reduce LDS: 4096 slots x 28 B
constexpr uint32_t kTileMin = 8192;
constexpr uint32_t kMaxTiles = 1024;
constexpr int kReduceThreads = 256;

struct Plan {
    uint32_t log2_bins, nbins, bin_shift, bin_slots, ntiles, tile;
    size_t off_h, off_tot, off_start, off_rec, bytes;
};

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

Plan make_plan(uint32_t n, uint32_t log2_slots) {
    Plan p;
    p.log2_bins = log2_slots > kLog2MinBinSlots ? log2_slots - kLog2MinBinSlots : 0;
    if (p.log2_bins > kLog2MaxBins) p.log2_bins = kLog2MaxBins;
    p.nbins = 1u << p.log2_bins;
    p.bin_shift = log2_slots - p.log2_bins;
    p.bin_slots = 1u << p.bin_shift;
    uint32_t nt = (n + kTileMin - 1) / kTileMin;
    if (nt > kMaxTiles) nt = kMaxTiles;
    if (nt == 0) nt = 1;
    p.ntiles = nt;
    p.tile = ((n + nt - 1) / nt + kT - 1) / kT * kT;
    p.off_h = 0;
    p.off_tot = align256((size_t)p.ntiles * p.nbins * 4);
    p.off_start = p.off_tot + align256((size_t)p.nbins * 4);
    p.off_rec = p.off_start + align256((size_t)p.nbins * 4);
    p.bytes = p.off_rec + align256((size_t)n * 16) + 256;
    return p;
}

// Probe / claim like find_or_claim, without the occupancy bit (set by the
// reduce pass, which owns the bitmap words of its bin).
__device__ __forceinline__ uint32_t claim(const Tab &t, uint64_t key) {
    const uint32_t f = fingerprint_of(key);
    uint32_t s = home_of(key, t.mask);
    for (uint32_t d = 0; d < t.max_probe; ++d) {
        uint32_t *pfp = &t.cell[s].fp;
        uint32_t cur = load_fp_probe(pfp);
        if (cur == 0) {
            uint32_t expected = 0;
            if (__hip_atomic_compare_exchange_strong(pfp, &expected, f, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                t.key[s] = key;
                return s;
            }
            cur = expected;
        }
        if (cur == f) return s;
        s = (s + 1) & t.mask;
    }
    return kNoSlot;
}

__global__ __launch_bounds__(kT) void claim_kernel(Tab t, const uint64_t *__restrict__ key,
                                                   const float *__restrict__ r, const float *__restrict__ g,
                                                   const float *__restrict__ b, uint8_t *__restrict__ flags,
                                                   uint32_t *__restrict__ slot_out, uint32_t n, uint32_t tile,
                                                   uint32_t nbins, uint32_t bin_shift, uint32_t *__restrict__ H) {
    extern __shared__ uint32_t hist[];
    for (uint32_t k = threadIdx.x; k < nbins; k += kT) hist[k] = 0;
    __syncthreads();
    const uint32_t i0 = blockIdx.x * tile;
    const uint32_t i1 = min(n, i0 + tile);
    uint32_t ovf = 0;
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += kT) {
        uint8_t fl = flags[i];
        const uint8_t fl0 = fl;
        uint32_t slot = kNoSlot;
        if (fl == 0) {
            int64_t q0, q1, q2;
            fl = fixed_point(r[i], g[i], b[i], t.frac_bits, q0, q1, q2);
        }
        if (fl == 0) {
            slot = claim(t, key[i]);
            if (slot == kNoSlot) {
                fl = PF_V_OVERFLOW;
                ++ovf;
            } else {
                atomicAdd(&hist[slot >> bin_shift], 1u);
            }
        }
        if (fl != fl0) flags[i] = fl;
        slot_out[i] = slot;
    }
    if (ovf) add_u64(&t.stats[PF_STAT_PART_OVF + (blockIdx.x & 15)], ovf);
    __syncthreads();
    uint32_t *row = H + (size_t)blockIdx.x * nbins;
    for (uint32_t k = threadIdx.x; k < nbins; k += kT) row[k] = hist[k];
}

// Per bin: exclusive running offset over the tiles (in place), bin total.
__global__ __launch_bounds__(256) void colscan_kernel(uint32_t *__restrict__ H, uint32_t ntiles, uint32_t nbins,
                                                      uint32_t *__restrict__ total) {
    const uint32_t bin = blockIdx.x * 256 + threadIdx.x;
    if (bin >= nbins) return;
    uint32_t run = 0;
    for (uint32_t t = 0; t < ntiles; ++t) {
        const uint32_t c = H[(size_t)t * nbins + bin];
        H[(size_t)t * nbins + bin] = run;
        run += c;
    }
    total[bin] = run;
}

// Exclusive scan of the bin totals (one workgroup, nbins <= 8192).
__global__ __launch_bounds__(1024) void binscan_kernel(const uint32_t *__restrict__ total, uint32_t nbins,
                                                       uint32_t *__restrict__ start) {
    __shared__ uint32_t part[1024];
    const uint32_t per = (nbins + 1023) / 1024;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t local = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < nbins) local += total[b0 + k];
    part[threadIdx.x] = local;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 partial sums
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - local;  // exclusive
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < nbins) {
            start[b0 + k] = run;
            run += total[b0 + k];
        }
}

__global__ __launch_bounds__(kT) void scatter_kernel(const float *__restrict__ r, const float *__restrict__ g,
                                                     const float *__restrict__ b, const uint8_t *__restrict__ flags,
                                                     const uint32_t *__restrict__ slot, uint32_t n, uint32_t tile,
                                                     uint32_t nbins, uint32_t bin_shift,
                                                     const uint32_t *__restrict__ H,
                                                     const uint32_t *__restrict__ start, uint4 *__restrict__ rec) {
    extern __shared__ uint32_t cursor[];
    const uint32_t *row = H + (size_t)blockIdx.x * nbins;
    for (uint32_t k = threadIdx.x; k < nbins; k += kT) cursor[k] = start[k] + row[k];
    __syncthreads();
    const uint32_t i0 = blockIdx.x * tile;
    const uint32_t i1 = min(n, i0 + tile);
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += kT) {
        if (flags[i] != 0) continue;
        const uint32_t s = slot[i];
        const uint32_t pos = atomicAdd(&cursor[s >> bin_shift], 1u);
        rec[pos] = make_uint4(s, __float_as_uint(r[i]), __float_as_uint(g[i]), __float_as_uint(b[i]));
    }
}

// One workgroup per bin: LDS sums over its records, then the exclusive
// owner adds them to the cells and sets the occupancy bits of its words.
__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(Tab t, const uint4 *__restrict__ rec,
                                                                const uint32_t *__restrict__ start,
                                                                const uint32_t *__restrict__ total,
                                                                uint32_t bin_slots) {
    extern __shared__ unsigned long long lds[];
    unsigned long long *sum0 = lds, *sum1 = lds + bin_slots, *sum2 = lds + 2 * bin_slots;
    uint32_t *cnt = reinterpret_cast<uint32_t *>(lds + 3 * bin_slots);
    const uint32_t bin = blockIdx.x;
    const uint32_t base = bin * bin_slots;
    for (uint32_t k = threadIdx.x; k < bin_slots; k += kReduceThreads) {
        sum0[k] = 0;
        sum1[k] = 0;
        sum2[k] = 0;
        cnt[k] = 0;
    }
    __syncthreads();
    const uint32_t j0 = start[bin], j1 = j0 + total[bin];
    for (uint32_t j = j0 + threadIdx.x; j < j1; j += kReduceThreads) {
        const uint4 e = rec[j];
        const uint32_t loc = e.x - base;
        int64_t q0, q1, q2;
        fixed_point(__uint_as_float(e.y), __uint_as_float(e.z), __uint_as_float(e.w), t.frac_bits, q0, q1, q2);
        atomicAdd(&sum0[loc], (unsigned long long)q0);
        atomicAdd(&sum1[loc], (unsigned long long)q1);
        atomicAdd(&sum2[loc], (unsigned long long)q2);
        atomicAdd(&cnt[loc], 1u);
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < bin_slots; k += kReduceThreads) {
        const uint32_t c = cnt[k];
        if (c == 0) continue;
        pf_cell *cell = t.cell + base + k;
        cell->count += c;
        cell->sum[0] = (int64_t)((uint64_t)cell->sum[0] + sum0[k]);
        cell->sum[1] = (int64_t)((uint64_t)cell->sum[1] + sum1[k]);
        cell->sum[2] = (int64_t)((uint64_t)cell->sum[2] + sum2[k]);
    }
    // occupancy words of this bin (bins hold >= 32 slots, or the whole table)
    const uint32_t words = (bin_slots + 31) / 32;
    for (uint32_t w = threadIdx.x; w < words; w += kReduceThreads) {
        uint32_t bits = 0;
        for (uint32_t k = 0; k < 32 && w * 32 + k < bin_slots; ++k) bits |= (cnt[w * 32 + k] != 0 ? 1u : 0u) << k;
        if (bits) t.occ[(base >> 5) + w] |= bits;
    }
}

}  // namespace binned

size_t binned_workspace_bytes(uint32_t n, uint32_t log2_slots) {
    if (log2_slots > binned::kMaxLog2Slots) return 0;
    return binned::make_plan(n, log2_slots).bytes;
}

hipError_t launch_insert_binned(const Tab &t, const uint64_t *key, const float *r, const float *g, const float *b,
                                uint8_t *flags, uint32_t *slot_out, uint32_t n, void *ws, hipStream_t st) {
    using namespace binned;
    const uint32_t log2_slots = 32 - __builtin_clz(t.mask + 1) - 1;
    const Plan p = make_plan(n, log2_slots);
    char *base = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(ws) + 255) / 256 * 256);
    uint32_t *H = reinterpret_cast<uint32_t *>(base + p.off_h);
    uint32_t *tot = reinterpret_cast<uint32_t *>(base + p.off_tot);
    uint32_t *start = reinterpret_cast<uint32_t *>(base + p.off_start);
    uint4 *rec = reinterpret_cast<uint4 *>(base + p.off_rec);
    const size_t hist_lds = (size_t)p.nbins * 4;
    const size_t red_lds = (size_t)p.bin_slots * 28;
    static bool attrs = false;  // dynamic LDS above 64 KB needs the attribute, set once per function
    if (!attrs) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(reduce_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)(4096 * 28));
        if (e != hipSuccess) return e;
        attrs = true;
    }
    claim_kernel<<<p.ntiles, kT, hist_lds, st>>>(t, key, r, g, b, flags, slot_out, n, p.tile, p.nbins, p.bin_shift,
                                                 H);
    colscan_kernel<<<(p.nbins + 255) / 256, 256, 0, st>>>(H, p.ntiles, p.nbins, tot);
    binscan_kernel<<<1, 1024, 0, st>>>(tot, p.nbins, start);
    scatter_kernel<<<p.ntiles, kT, hist_lds, st>>>(r, g, b, flags, slot_out, n, p.tile, p.nbins, p.bin_shift, H,
                                                   start, rec);
    reduce_kernel<<<p.nbins, kReduceThreads, red_lds, st>>>(t, rec, start, tot, p.bin_slots);
    return hipGetLastError();
}

}  // namespace pfk
