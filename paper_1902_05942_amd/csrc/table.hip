// Hash table kernels for gfx950: initialisation, clearing, accumulation with
// linear probing (Section 3.2), lookup of cell averages, and the table
// statistics.  Occupied slots are recorded in a bitmap (one atomicOr per
// claimed slot, spread over 2^m/32 words) so that no kernel updates a
// shared counter per cell.
#include <type_traits>

#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

constexpr uint32_t kScanGrid = 2048;  // blocks of the grid-stride kernels over the bitmap

// ----------------------------------------------------------------- init
__global__ __launch_bounds__(kBlock) void table_init_kernel(uint4 *__restrict__ cells16, uint64_t n16,
                                                            uint32_t *__restrict__ occ, uint32_t nwords,
                                                            unsigned long long *__restrict__ stats) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    for (uint64_t j = tid; j < n16; j += stride) cells16[j] = make_uint4(0, 0, 0, 0);
    for (uint64_t j = tid; j < nwords; j += stride) occ[j] = 0;
    if (blockIdx.x == 0 && threadIdx.x < PF_STATS_LEN) stats[threadIdx.x] = 0;
}
static_assert(PF_STATS_LEN <= kBlock, "one block zeroes the statistics");

hipError_t launch_table_init(const Tab &t, hipStream_t st) {
    const uint64_t n16 = ((uint64_t)t.mask + 1) * PF_SLOT_BYTES / sizeof(uint4);
    uint64_t blocks = (n16 + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    table_init_kernel<<<(uint32_t)blocks, kBlock, 0, st>>>(reinterpret_cast<uint4 *>(t.rec), n16, t.occ,
                                                           t.nwords(), t.stats);
    return hipGetLastError();
}

// ----------------------------------------------------------------- clear
// Zeroes the cells whose occupancy bit is set and the bitmap words, as
// workgroup `blk` of `nblk` taking every nblk-th range of bitmap words;
// workgroup 0 zeroes the statistics (no kernel reads them here).
__device__ __forceinline__ void clear_part(const Tab &t, uint32_t blk, uint32_t nblk) {
    const uint32_t nwords = t.nwords();
    const uint32_t stride = nblk * kBlock;
    for (uint32_t j = blk * kBlock + threadIdx.x; j < nwords; j += stride) {
        uint32_t w = t.occ[j];
        if (w == 0) continue;
        t.occ[j] = 0;
        while (w) {
            const uint32_t b = __builtin_ctz(w);
            w &= w - 1;
            uint4 *c = t.words_at(j * 32 + b);
            c[0] = make_uint4(0, 0, 0, 0);
            c[1] = make_uint4(0, 0, 0, 0);
        }
    }
    if (blk == 0 && threadIdx.x < PF_STATS_LEN) t.stats[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kBlock) void clear_kernel(Tab t) { clear_part(t, blockIdx.x, gridDim.x); }

static uint32_t scan_blocks(uint32_t items) {
    const uint32_t b = (items + kBlock - 1) / kBlock;
    return b < kScanGrid ? (b ? b : 1) : kScanGrid;
}

hipError_t launch_clear(const Tab &t, hipStream_t st) {
    clear_kernel<<<scan_blocks(t.nwords()), kBlock, 0, st>>>(t);
    return hipGetLastError();
}

// ----------------------------------------------------------------- insert
// V = int64_t: fixed-point sums; V = float: binary32 sums (PF_SUMS_FLOAT32).
template <bool kAgg, typename V>
__global__ __launch_bounds__(kBlock) void insert_kernel(Tab t, const uint64_t *__restrict__ key,
                                                        const float *__restrict__ r, const float *__restrict__ g,
                                                        const float *__restrict__ b, uint8_t *__restrict__ flags,
                                                        uint32_t *__restrict__ slot_out, uint32_t n, uint32_t agg) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool in = i < n;
    uint8_t fl = in ? flags[i] : (uint8_t)PF_V_INVALID;
    const uint8_t fl0 = fl;
    V q0 = 0, q1 = 0, q2 = 0;
    if (fl == 0) {
        if constexpr (std::is_same<V, float>::value)
            fl = float_contribution(r[i], g[i], b[i], q0, q1, q2);
        else
            fl = fixed_point(r[i], g[i], b[i], t.frac_bits, q0, q1, q2);
    }
    uint32_t slot = kNoSlot;
    if (fl == 0) {
        slot = find_or_claim(t, key[i]);
        if (slot == kNoSlot) {
            fl = PF_V_OVERFLOW;
            add_u64(&t.stats[PF_STAT_PART_OVF + (blockIdx.x & 15)], 1ull);
        }
    }
    if (in && fl != fl0) flags[i] = fl;
    if (in && slot_out) slot_out[i] = slot;
    if constexpr (!kAgg) {
        if (slot != kNoSlot) accumulate(t, slot, 1, q0, q1, q2);
    } else {
        __shared__ AggLds<kBlock> L;
        accumulate_group<kBlock, V>(t, L, agg, slot, q0, q1, q2);
    }
}

template <typename V>
static void launch_insert_t(const Tab &t, const uint64_t *key, const float *r, const float *g, const float *b,
                            uint8_t *flags, uint32_t *slot_out, uint32_t n, uint32_t agg_width, hipStream_t st) {
    const uint32_t blocks = (n + kBlock - 1) / kBlock;
    if (agg_width <= 1)
        insert_kernel<false, V><<<blocks, kBlock, 0, st>>>(t, key, r, g, b, flags, slot_out, n, 1);
    else
        insert_kernel<true, V><<<blocks, kBlock, 0, st>>>(t, key, r, g, b, flags, slot_out, n, agg_width);
}

hipError_t launch_insert(const Tab &t, const uint64_t *key, const float *r, const float *g, const float *b,
                         uint8_t *flags, uint32_t *slot_out, uint32_t n, uint32_t agg_width, hipStream_t st) {
    if (t.fsum)
        launch_insert_t<float>(t, key, r, g, b, flags, slot_out, n, agg_width, st);
    else
        launch_insert_t<int64_t>(t, key, r, g, b, flags, slot_out, n, agg_width, st);
    return hipGetLastError();
}

// ----------------------------------------------------------------- query
template <bool kBlend>
__device__ __forceinline__ void query_one(const Tab &t, uint32_t i, const uint64_t *__restrict__ key,
                                          const uint32_t *__restrict__ slot_in, const float *r, const float *g,
                                          const float *b, const uint8_t *__restrict__ flags, float *ro, float *go,
                                          float *bo, uint32_t *__restrict__ count_out, bool inplace) {
    // the flag and the slot are loaded together; the flag decides
    const uint8_t fl = flags[i];
    uint32_t slot = slot_in ? slot_in[i] : kNoSlot;
    if (fl != 0)
        slot = kNoSlot;
    else if (!slot_in)
        slot = find_slot(t, key[i]);
    query_vertex<kBlend>(t, slot, i, r, g, b, ro, go, bo, count_out, inplace);
}

template <bool kBlend>
__global__ __launch_bounds__(kBlock) void query_kernel(Tab t, const uint64_t *__restrict__ key,
                                                       const uint32_t *__restrict__ slot_in, const float *r,
                                                       const float *g, const float *b,
                                                       const uint8_t *__restrict__ flags, uint32_t n, float *ro,
                                                       float *go, float *bo, uint32_t *__restrict__ count_out,
                                                       bool inplace) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    query_one<kBlend>(t, i, key, slot_in, r, g, b, flags, ro, go, bo, count_out, inplace);
}

// The lookup in t and, in the same launch, the clear of another table: the
// first `cblocks` workgroups empty `clr` (dispatched first, their scattered
// stores overlap the lookup's gathers), the others look up one vertex per
// lane.
template <bool kBlend>
__global__ __launch_bounds__(kBlock) void query_clear_kernel(Tab t, const uint64_t *__restrict__ key,
                                                             const uint32_t *__restrict__ slot_in, const float *r,
                                                             const float *g, const float *b,
                                                             const uint8_t *__restrict__ flags, uint32_t n, float *ro,
                                                             float *go, float *bo, uint32_t *__restrict__ count_out,
                                                             bool inplace, Tab clr, uint32_t cblocks) {
    if (blockIdx.x < cblocks) {
        clear_part(clr, blockIdx.x, cblocks);
        return;
    }
    const uint32_t i = (blockIdx.x - cblocks) * kBlock + threadIdx.x;
    if (i >= n) return;
    query_one<kBlend>(t, i, key, slot_in, r, g, b, flags, ro, go, bo, count_out, inplace);
}

hipError_t launch_query(const Tab &t, const uint64_t *key, const uint32_t *slot, const float *r, const float *g,
                        const float *b, const uint8_t *flags, uint32_t n, bool use_blend, float *ro, float *go,
                        float *bo, uint32_t *count_out, hipStream_t st) {
    const uint32_t blocks = (n + kBlock - 1) / kBlock;
    const bool inplace = (ro == r) && (go == g) && (bo == b);
    if (use_blend)
        query_kernel<true><<<blocks, kBlock, 0, st>>>(t, key, slot, r, g, b, flags, n, ro, go, bo, count_out, inplace);
    else
        query_kernel<false><<<blocks, kBlock, 0, st>>>(t, key, slot, r, g, b, flags, n, ro, go, bo, count_out, inplace);
    return hipGetLastError();
}

hipError_t launch_query_clear(const Tab &t, const uint64_t *key, const uint32_t *slot, const float *r, const float *g,
                              const float *b, const uint8_t *flags, uint32_t n, bool use_blend, float *ro, float *go,
                              float *bo, uint32_t *count_out, const Tab &clr, hipStream_t st) {
    const uint32_t cblocks = scan_blocks(clr.nwords());
    const uint32_t blocks = cblocks + (n + kBlock - 1) / kBlock;
    const bool inplace = (ro == r) && (go == g) && (bo == b);
    if (use_blend)
        query_clear_kernel<true><<<blocks, kBlock, 0, st>>>(t, key, slot, r, g, b, flags, n, ro, go, bo, count_out,
                                                           inplace, clr, cblocks);
    else
        query_clear_kernel<false><<<blocks, kBlock, 0, st>>>(t, key, slot, r, g, b, flags, n, ro, go, bo, count_out,
                                                            inplace, clr, cblocks);
    return hipGetLastError();
}

// ----------------------------------------------------------------- statistics
// Zeroes the derived counters and folds the partial counters.
__global__ void stats_zero_kernel(unsigned long long *stats) {
    const uint32_t k = threadIdx.x;
    if (k == PF_STAT_USED || k == PF_STAT_DISP || (k >= PF_STAT_HIST && k < PF_STAT_HIST + 65)) stats[k] = 0;
    if (k == PF_STAT_OVERFLOW) {
        unsigned long long v = 0;
        for (int j = 0; j < 16; ++j) v += stats[PF_STAT_PART_OVF + j];
        stats[k] = v;
    }
    if (k == PF_STAT_TEMPORAL_HIT) {
        unsigned long long v = 0;
        for (int j = 0; j < 32; ++j) v += stats[PF_STAT_PART_HIT + j];
        stats[k] = v;
    }
}

// USED, DISP and HIST from the bitmap and the stored keys: block-local sums
// in LDS, then one device atomic per non-zero block total.
__global__ __launch_bounds__(kBlock) void stats_kernel(Tab t) {
    __shared__ unsigned long long s_used, s_disp;
    __shared__ unsigned long long s_hist[65];
    if (threadIdx.x == 0) {
        s_used = 0;
        s_disp = 0;
    }
    if (threadIdx.x < 65) s_hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t nwords = t.nwords();
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < nwords; j += stride) {
        uint32_t w = t.occ[j];
        if (w) atomicAdd(&s_used, (unsigned long long)__popc(w));
        while (w) {
            const uint32_t s = j * 32 + __builtin_ctz(w);
            w &= w - 1;
            const uint32_t d = (s - home_of(t.key_at(s), t.mask)) & t.mask;
            atomicAdd(&s_disp, (unsigned long long)d);
            atomicAdd(&s_hist[d < 64 ? d : 64], 1ull);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_used) add_u64(&t.stats[PF_STAT_USED], s_used);
        if (s_disp) add_u64(&t.stats[PF_STAT_DISP], s_disp);
    }
    if (threadIdx.x < 65 && s_hist[threadIdx.x]) add_u64(&t.stats[PF_STAT_HIST + threadIdx.x], s_hist[threadIdx.x]);
}

hipError_t launch_stats(const Tab &t, hipStream_t st) {
    stats_zero_kernel<<<1, PF_STATS_LEN, 0, st>>>(t.stats);
    stats_kernel<<<scan_blocks(t.nwords()), kBlock, 0, st>>>(t);
    return hipGetLastError();
}

}  // namespace pfk
