// Many views in one persistent launch on gfx950.  A cooperative grid of
// resident workgroups walks four phases -- clear, keys + insert, temporal,
// lookup -- separated by grid-wide barriers.  Within a phase the work items
// of all views (chunks of bitmap words, vertices or slots) are dealt to the
// workgroups round-robin, so small and large views share the whole chip.
// The per-vertex and per-cell arithmetic is that of the single-view kernels
// (pf_ops.h).
#include "pf_kernels.h"
#include "pf_merge.h"
#include "pf_ops.h"

namespace pfk {

namespace views {

constexpr int kIters = 8;            // block-sized steps per work item
constexpr int kSubCounters = 64;     // first level of the grid barrier
constexpr int kCounterStride = 16;   // uint32 words between counters (64 B)

struct Barrier {
    uint32_t *status;   // [0] non-zero once a wait has timed out
    uint32_t *sub;      // kSubCounters arrival counters, kCounterStride apart
    uint32_t *rel;      // kSubCounters release flags, kCounterStride apart
    uint32_t *top;      // sub-groups arrived
    uint64_t limit;     // wall-clock ticks a wait may last
};

// Reads a counter at the coherence point with a read-modify-write that adds
// 0: loads may be served by an XCD's L2, which does not see atomics made
// elsewhere.  The zero is hidden from the optimiser, which would otherwise
// turn the idempotent read-modify-write back into a plain load.
__device__ __forceinline__ uint32_t poll(uint32_t *p) {
    uint32_t zero = 0;
    asm volatile("" : "+v"(zero));
    return __hip_atomic_fetch_add(p, zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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

// Grid-wide barrier number `epoch` (1, 2, 3 ...).  A workgroup arrives at
// one of 64 sub-counters; the last arrival of a sub-group advances the top
// counter, waits for all sub-groups, then raises its sub-group's release
// flag, on which the other members wait.  So at most ~64 workgroups poll any
// one address.  Release/acquire fences make the phase's writes visible
// across XCDs.  Every wait is bounded in wall-clock time; a timed-out wait
// sets the status word and returns false (the workgroup then leaves).
__device__ bool grid_barrier(const Barrier &bar, uint32_t epoch) {
    __shared__ uint32_t s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t G = gridDim.x;
        const uint32_t nsub = G < (uint32_t)kSubCounters ? G : (uint32_t)kSubCounters;
        const uint32_t sub = blockIdx.x % nsub;
        const uint32_t in_sub = (G - sub + nsub - 1) / nsub;  // workgroups of this sub-group
        const uint32_t old = __hip_atomic_fetch_add(bar.sub + sub * kCounterStride, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        uint32_t ok = 1;
        if (old + 1 == epoch * in_sub) {
            __hip_atomic_fetch_add(bar.top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while (poll(bar.top) < epoch * nsub) {
                if (wall_clock64() - t0 > bar.limit) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
            __hip_atomic_fetch_max(bar.rel + sub * kCounterStride, ok ? epoch : 0xffffffffu, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            for (;;) {
                const uint32_t r = poll(bar.rel + sub * kCounterStride);
                if (r == 0xffffffffu) {
                    ok = 0;
                    break;
                }
                if (r >= epoch) break;
                if (wall_clock64() - t0 > bar.limit) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        if (!ok) {
            __hip_atomic_fetch_or(bar.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(bar.status + 2, poll(bar.top), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(bar.status + 3, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __threadfence();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// LDS merge table of the insert phase: a window of agg_width consecutive
// vertices (block .. kIters * block) merges into at most min(agg_width,
// 4 * block, 1536) entries (the table stays in static LDS and small
// workgroups keep their residency); a vertex that finds no room goes alone.
template <int B>
constexpr uint32_t kMergeCap = 4 * B < 1536 ? 4 * B : 1536;

template <int B>
struct Lds {
    unsigned long long mkey[kMergeCap<B>];
    unsigned long long ms0[kMergeCap<B>], ms1[kMergeCap<B>], ms2[kMergeCap<B>];
    uint32_t mcnt[kMergeCap<B>];           // count, then the group's slot
    uint32_t first[4][PF_MAX_VIEWS + 1];  // per phase: first global item of each view
    uint32_t hits;
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

// At least kWavesPerSimd waves of this kernel fit a SIMD (the compiler
// keeps the registers within that), which bounds the resident workgroups
// from below independently of the occupancy query.
constexpr int kWavesPerSimd = 4;

template <int B>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd))) void views_kernel(
    const pf_view *__restrict__ views, uint32_t nviews, uint32_t agg, Barrier bar) {
    __shared__ Lds<B> L;
    constexpr uint32_t kItem = (uint32_t)B * kIters;
    // work items per view and phase: 0 clear (B bitmap words), 1 keys +
    // insert (8 x B vertices), 2 temporal (B bitmap words), 3 lookup (8 x B
    // vertices)
    if (threadIdx.x == 0) {
        uint32_t acc[4] = {0, 0, 0, 0};
        for (uint32_t v = 0; v < nviews; ++v) {
            const pf_view &d = views[v];
            const uint32_t slots = 1u << d.cur.log2_slots;
            const uint32_t words = (slots + 31) / 32;
            const uint32_t items[4] = {(words + B - 1) / B, (d.n + kItem - 1) / kItem,
                                       d.temporal ? (words + B - 1) / B : 0u, (d.n + kItem - 1) / kItem};
            for (int p = 0; p < 4; ++p) {
                L.first[p][v] = acc[p];
                acc[p] += items[p];
            }
        }
        for (int p = 0; p < 4; ++p) L.first[p][nviews] = acc[p];
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

    // ---- phase 0: clear the current tables
    for (uint32_t it = blockIdx.x; it < L.first[0][nviews]; it += G) {
        uint32_t v, local;
        item_of(L, 0, nviews, it, v, local);
        const Tab t = to_tab(views[v].cur);
        const uint32_t j = local * B + threadIdx.x;  // one bitmap word per lane
        if (j < t.nwords()) {
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
        if (local == 0)
            for (uint32_t k = threadIdx.x; k < PF_STATS_LEN; k += B) t.stats[k] = 0;
    }
    if (!grid_barrier(bar, 1)) return;
    stamp(1);

    // ---- phase 1: keys and insertion.  agg == 0: one claim and one set of
    // device atomics per vertex.  Otherwise each window of agg consecutive
    // vertices (a power of two, block <= agg <= kIters * block) merges by key
    // in LDS, then every group claims its cell once and adds its count and
    // sums with one set of atomics.
    const uint32_t kCap = agg < kMergeCap<B> ? agg : kMergeCap<B>;
    const uint32_t per = agg / B;  // vertices per lane and window (1, 2, 4 or 8)
    for (uint32_t it = blockIdx.x; it < L.first[1][nviews]; it += G) {
        uint32_t v, local;
        item_of(L, 1, nviews, it, v, local);
        const pf_view &d = views[v];
        const Tab t = to_tab(d.cur);
        const float inv_s = 1.0f / d.kp.s;
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
                d.key[i] = key;
                d.vflags[i] = fl;
                d.slot[i] = slot;
            }
            continue;
        }
        for (uint32_t sub = 0; sub < (uint32_t)kIters / per; ++sub) {
            const uint32_t base = local * kItem + sub * agg;
            if (base >= d.n) break;  // uniform across the workgroup
            for (uint32_t j = threadIdx.x; j < kCap; j += B) {
                L.mkey[j] = kEmpty;
                L.ms0[j] = 0;
                L.ms1[j] = 0;
                L.ms2[j] = 0;
                L.mcnt[j] = 0;
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
                if (i < d.n) d.key[i] = k;
                const int e = merge_into_lds<false>(L.mkey, L.ms0, L.ms1, L.ms2, L.mcnt, kCap, f == 0, k, q0, q1, q2);
                fv |= (uint64_t)f << (8 * u);
                const uint64_t eb = (uint64_t)(uint16_t)e << (16 * (u & 3));
                if (u < 4)
                    ev[0] |= eb;
                else
                    ev[1] |= eb;
            }
            __syncthreads();
            for (uint32_t j = threadIdx.x; j < kCap; j += B) {
                const unsigned long long kk = L.mkey[j];
                if (kk == kEmpty) continue;
                const uint32_t c = L.mcnt[j];
                const uint32_t slot = find_or_claim(t, kk);
                if (slot != kNoSlot)
                    accumulate(t, slot, c, (int64_t)L.ms0[j], (int64_t)L.ms1[j], (int64_t)L.ms2[j]);
                else
                    add_u64(&t.stats[PF_STAT_PART_OVF + (blockIdx.x & 15)], (unsigned long long)c);
                L.mcnt[j] = slot;
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
                        slot = L.mcnt[e];
                    } else {  // no room in the LDS table: on its own
                        uint64_t k;
                        int64_t q0, q1, q2;
                        view_vertex(d, t, inv_s, i, k, q0, q1, q2);
                        slot = find_or_claim(t, k);
                        if (slot != kNoSlot)
                            accumulate(t, slot, 1, q0, q1, q2);
                        else
                            add_u64(&t.stats[PF_STAT_PART_OVF + (blockIdx.x & 15)], 1ull);
                    }
                    if (slot == kNoSlot) fl = PF_V_OVERFLOW;
                }
                d.vflags[i] = fl;
                d.slot[i] = slot;
            }
            __syncthreads();  // the table is cleared for the next sub-chunk
        }
    }
    if (!grid_barrier(bar, 2)) return;
    stamp(2);

    // ---- phase 2: temporal values
    for (uint32_t it = blockIdx.x; it < L.first[2][nviews]; it += G) {
        uint32_t v, local;
        item_of(L, 2, nviews, it, v, local);
        const pf_view &d = views[v];
        const Tab cur = to_tab(d.cur);
        const bool has_prev = d.prev.cell != nullptr;
        const Tab prev = has_prev ? to_tab(d.prev) : cur;
        const float alpha = d.alpha_old, beta = 1.0f - d.alpha_old;
        // an item is one word per lane: a word holds 32 slots, so finer items
        // than the other phases' keep every workgroup busy
        const uint32_t j = local * B + threadIdx.x;
        uint32_t hits = 0;
        if (j < cur.nwords()) {
            if (has_prev)
                hits = temporal_word<true, false, 2>(cur, prev, j, alpha, beta, 0u);
            else
                temporal_word<false, false, 2>(cur, prev, j, alpha, beta, 0u);
        }
        if (has_prev) {
            if (threadIdx.x == 0) L.hits = 0;
            __syncthreads();
            if (hits) atomicAdd(&L.hits, hits);
            __syncthreads();
            if (threadIdx.x == 0 && L.hits) add_u64(&cur.stats[PF_STAT_PART_HIT + (blockIdx.x & 31)], L.hits);
            __syncthreads();
        }
    }
    if (!grid_barrier(bar, 3)) return;
    stamp(3);

    // ---- phase 3: lookup
    for (uint32_t it = blockIdx.x; it < L.first[3][nviews]; it += G) {
        uint32_t v, local;
        item_of(L, 3, nviews, it, v, local);
        const pf_view &d = views[v];
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

template <int B>
hipError_t launch_b(const pf_view *views, uint32_t nviews, uint32_t agg, uint32_t per_cu, uint32_t *ws,
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
        const int by_waves = 4 * kWavesPerSimd * 64 / B > 0 ? 4 * kWavesPerSimd * 64 / B : 1;
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
    Barrier bar;
    bar.status = ws;
    bar.sub = ws + kCounterStride;
    bar.rel = ws + kCounterStride * (1 + kSubCounters);
    bar.top = ws + kCounterStride * (1 + 2 * kSubCounters);
    bar.limit = 2 * ticks_per_s;  // a phase never takes seconds
    const uint32_t words = kCounterStride * (2 + 2 * kSubCounters);
    views_reset_kernel<<<1, 256, 0, st>>>(ws, words);
    const uint32_t per = (per_cu == 0 || per_cu > (uint32_t)resident) ? (uint32_t)resident : per_cu;
    uint32_t grid = per * (uint32_t)cus;
    void *args[] = {(void *)&views, (void *)&nviews, (void *)&agg, (void *)&bar};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(views_kernel<B>), dim3(grid), dim3(B), args, 0,
                                      st);
}

}  // namespace views

size_t views_counter_bytes() { return sizeof(uint32_t) * views::kCounterStride * (2 * views::kSubCounters + 2); }

hipError_t launch_views(const pf_view *views_dev, uint32_t nviews, uint32_t block, uint32_t agg, uint32_t per_cu,
                        uint32_t *ws, hipStream_t st) {
    switch (block) {
        case 64: return views::launch_b<64>(views_dev, nviews, agg, per_cu, ws, st);
        case 128: return views::launch_b<128>(views_dev, nviews, agg, per_cu, ws, st);
        case 256: return views::launch_b<256>(views_dev, nviews, agg, per_cu, ws, st);
        case 512: return views::launch_b<512>(views_dev, nviews, agg, per_cu, ws, st);
        case 1024: return views::launch_b<1024>(views_dev, nviews, agg, per_cu, ws, st);
        default: return hipErrorInvalidConfiguration;
    }
}

}  // namespace pfk
