// Memory-system probes that give the filter's rooflines measured
// denominators on the device at hand: streaming copy bandwidth, and the rate
// of random accesses of one granule (gather, scatter, the cell update's
// read-modify-write atomics, compare-and-swap) over a footprint the size of
// a table.  Indices come from fmix64 of (seed, access number), so every
// access is in bounds and independent of the data.
#include "pf_kernels.h"

namespace pfk {

namespace mb {

constexpr int kT = 256;

__device__ __forceinline__ uint64_t mix(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// dst[i] = src[i] over n 16-byte words, grid-stride
__global__ __launch_bounds__(kT) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * kT;
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// per thread `per` accesses to granules of `words` 16-byte words chosen at
// random among `mask + 1` granules; kind: 1 gather, 2 scatter, 3 cell
// read-modify-write (u32 + 3 x u64 atomic adds), 4 compare-and-swap
template <int kKind>
__global__ __launch_bounds__(kT) void random_kernel(uint4 *__restrict__ buf, uint64_t mask, uint32_t words,
                                                   uint32_t per, uint64_t seed, uint32_t *__restrict__ sink) {
    const uint64_t t = (uint64_t)blockIdx.x * kT + threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t k = 0; k < per; ++k) {
        const uint64_t g = mix(seed ^ (t * per + k)) & mask;
        uint4 *p = buf + g * words;
        if constexpr (kKind == 1) {
            for (uint32_t w = 0; w < words; ++w) acc += p[w].x ^ p[w].w;
        } else if constexpr (kKind == 2) {
            for (uint32_t w = 0; w < words; ++w) p[w] = make_uint4((uint32_t)t, k, w, 0);
        } else if constexpr (kKind == 3) {
            uint32_t *c = reinterpret_cast<uint32_t *>(p);
            unsigned long long *s = reinterpret_cast<unsigned long long *>(p);
            __hip_atomic_fetch_add(c + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(s + 1, 3ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(s + 2, 5ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(s + 3, 7ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t expected = 0;
            __hip_atomic_compare_exchange_strong(reinterpret_cast<uint32_t *>(p), &expected, (uint32_t)t | 1u,
                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            acc += expected;
        }
    }
    if constexpr (kKind == 1 || kKind == 4)
        if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads; practically never stores
}

}  // namespace mb

hipError_t launch_microbench(int kind, void *buf, uint64_t bytes, uint32_t grain, uint64_t accesses, uint64_t seed,
                             uint32_t *sink, hipStream_t st) {
    using namespace mb;
    if (kind == 0) {
        const uint64_t n = bytes / 2 / sizeof(uint4);
        uint4 *src = reinterpret_cast<uint4 *>(buf);
        copy_kernel<<<4096, kT, 0, st>>>(src, src + n, n);
        return hipGetLastError();
    }
    const uint32_t words = grain / 16;
    const uint64_t granules = bytes / grain;           // a power of two (checked by the caller)
    const uint32_t threads = 8192 * kT;
    const uint32_t per = (uint32_t)((accesses + threads - 1) / threads);
    uint4 *b = reinterpret_cast<uint4 *>(buf);
    switch (kind) {
        case 1: random_kernel<1><<<8192, kT, 0, st>>>(b, granules - 1, words, per, seed, sink); break;
        case 2: random_kernel<2><<<8192, kT, 0, st>>>(b, granules - 1, words, per, seed, sink); break;
        case 3: random_kernel<3><<<8192, kT, 0, st>>>(b, granules - 1, words, per, seed, sink); break;
        default: random_kernel<4><<<8192, kT, 0, st>>>(b, granules - 1, words, per, seed, sink); break;
    }
    return hipGetLastError();
}

}  // namespace pfk
