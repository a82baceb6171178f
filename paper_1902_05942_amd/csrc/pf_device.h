// Device-side building blocks of hashed path space filtering for gfx950.
//
// Everything here is inline and used by the kernels of this library only.
// All binary32 arithmetic is written as separate, individually rounded
// operations; translation units including this header are compiled with
// -ffp-contract=off and additionally request it below, so no multiply-add is
// ever fused and results are bit-reproducible against any IEEE binary32
// evaluation of the same expressions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf.h"

#pragma clang fp contract(off)

namespace pfk {

constexpr int kLevelMin = -16;
constexpr int kLevelMax = 15;
constexpr float kCellIndexLimit = 65536.0f;   // |x~| < 2^16
constexpr uint64_t kPosMask = (1ull << 56) - 1;  // key bits holding x~ and l'
constexpr uint32_t kNoSlot = 0xffffffffu;
constexpr int kBlock = 256;

// Level of detail of Algorithm 1: floor(log2 d) from the binary32 value
// d^2 = (dx*dx + dy*dy) + dz*dz.  The exponent field of d^2 is
// floor(log2 d^2) for normal numbers, and floor(e / 2) (arithmetic shift)
// is floor(log2 d).  Zero and subnormal d^2 give the lowest level, an
// infinite d^2 the highest.
__device__ __forceinline__ int level_of_detail(float cx, float cy, float cz, float x, float y, float z) {
    const float dx = cx - x;
    const float dy = cy - y;
    const float dz = cz - z;
    const float xx = dx * dx;
    const float yy = dy * dy;
    const float zz = dz * dz;
    const float d2 = (xx + yy) + zz;
    const int e = (int)((__float_as_uint(d2) >> 23) & 0xffu);
    int l = (e == 0) ? kLevelMin : ((e == 255) ? kLevelMax : ((e - 127) >> 1));
    l = l < kLevelMin ? kLevelMin : l;
    l = l > kLevelMax ? kLevelMax : l;
    return l;
}

// PCG32 (O'Neill 2014): 64-bit LCG, XSH-RR output, standard seeding.
struct Pcg32 {
    uint64_t state;
    uint64_t inc;

    __device__ __forceinline__ uint32_t next() {
        const uint64_t old = state;
        state = old * 6364136223846793005ull + inc;
        const uint32_t xs = (uint32_t)(((old >> 18) ^ old) >> 27);
        const uint32_t rot = (uint32_t)(old >> 59);
        return (xs >> rot) | (xs << ((32u - rot) & 31u));
    }

    __device__ __forceinline__ Pcg32(uint64_t initstate, uint64_t initseq) {
        state = 0;
        inc = (initseq << 1) | 1ull;
        next();
        state += initstate;
        next();
    }
};

// The first three outputs of PCG32 seeded with (initstate, base + i) for the
// vertices i of a launch, by jumping the LCG ahead instead of stepping it
// (Brown 1994, random number generation with arbitrary strides: k steps of
// x -> M x + c give M^k x + c (M^(k-1) + ... + 1) mod 2^64).  The standard
// seeding leaves the state S_0 = (inc + initstate) M + inc with
// inc = 2 (base + i) + 1, and output k is the XSH-RR permutation of
//   S_k = initstate M^(k+1) + G_(k+1) (2 (base + i) + 1),  G_j = 1 + M + .. + M^j,
// an affine function F_k + E_k i of i whose coefficients are the same for
// every vertex of the launch.  The outputs equal Pcg32's exactly.
struct PcgJump {
    static constexpr uint64_t kM = 6364136223846793005ull;
    static constexpr uint64_t kM2 = kM * kM, kM3 = kM2 * kM, kM4 = kM3 * kM;
    static constexpr uint64_t kG1 = 1ull + kM, kG2 = kG1 + kM2, kG3 = kG2 + kM3;
    uint64_t F[3], E[3];

    __host__ __device__ __forceinline__ PcgJump(uint64_t initstate, uint64_t base) {
        const uint64_t Mk[3] = {kM, kM2, kM3}, Gk[3] = {kG1, kG2, kG3};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            E[k] = 2ull * Gk[k];
            F[k] = initstate * Mk[k] + Gk[k] * (2ull * base + 1ull);
        }
    }

    __device__ __forceinline__ uint32_t output(int k, uint32_t i) const {
        const uint64_t old = F[k] + E[k] * (uint64_t)i;
        const uint32_t xs = (uint32_t)(((old >> 18) ^ old) >> 27);
        const uint32_t rot = (uint32_t)(old >> 59);
        return (xs >> rot) | (xs << ((32u - rot) & 31u));
    }
};

// floor of the binary32 quotient RN(x / h) that Algorithm 1 quantises, for
// h = s 2^l, given r = RN(1/s) 2^-l.  t = RN(x r) is within 2.0001 u |t| of
// the exact quotient y (u = 2^-24) and RN(y) within u |y| of y, so when no
// integer lies within 4 u |t| of t, floor(RN(y)) = floor(t); otherwise (or
// when t is not finite) the IEEE division decides.
__device__ __forceinline__ float floor_quotient(float x, float h, float r) {
    const float t = x * r;
    const float f = floorf(t);
    const float frac = t - f;
    const float m = 2.38418579e-7f * fabsf(t);  // 4 u |t|
    if (frac > m && 1.0f - frac > m) return f;
    return floorf(x / h);
}

// MurmurHash3 64-bit finaliser: the home index hash.
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// SplitMix64 output function: the fingerprint hash.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t home_of(uint64_t key, uint32_t mask) {
    return (uint32_t)(fmix64(key & kPosMask)) & mask;
}

__device__ __forceinline__ uint32_t fingerprint_of(uint64_t key) {
    const uint32_t f = (uint32_t)(splitmix64(key) >> 32);
    return f ? f : 1u;
}

__device__ __forceinline__ uint32_t normal_class(float c) {
    return (c > 0.0f) ? 1u : ((c < 0.0f) ? 2u : 0u);
}

// Cell average: (float)((double)sum * 2^-F / (double)count), one rounding
// of the quotient to binary32 after an exact scaling.
__device__ __forceinline__ float cell_average(int64_t sum, uint32_t count, int frac_bits) {
    const double s = ldexp((double)sum, -frac_bits);
    return (float)(s / (double)count);
}

// binary32 sum held in the low word of a cell's sum (PF_SUMS_FLOAT32)
__device__ __forceinline__ float *float_sum(pf_cell *c, int k) { return reinterpret_cast<float *>(&c->sum[k]); }
__device__ __forceinline__ float float_sum_value(int64_t word) { return __uint_as_float((uint32_t)(uint64_t)word); }

// Table handle passed to kernels by value.
static_assert(sizeof(pf_cell) == 32 && PF_SLOT_BYTES == 64, "slot record layout");

struct Tab {
    unsigned char *rec;  // slot records of PF_SLOT_BYTES: cell at 0, key at 32, temporal value at 48
    uint32_t *occ;
    unsigned long long *stats;
    uint32_t mask;
    uint32_t max_probe;
    int32_t frac_bits;
    uint32_t fsum;  // 1: binary32 sums in the low word of each sum (PF_SUMS_FLOAT32)

    __device__ __forceinline__ pf_cell &cell_at(uint32_t s) const {
        return *reinterpret_cast<pf_cell *>(rec + (size_t)s * PF_SLOT_BYTES);
    }
    __device__ __forceinline__ uint64_t &key_at(uint32_t s) const {
        return *reinterpret_cast<uint64_t *>(rec + (size_t)s * PF_SLOT_BYTES + 32);
    }
    __device__ __forceinline__ float4 &blend_at(uint32_t s) const {
        return *reinterpret_cast<float4 *>(rec + (size_t)s * PF_SLOT_BYTES + 48);
    }
    // slot s as 16-byte words: [0], [1] the cell, [2] the key (and padding), [3] the temporal value
    __device__ __forceinline__ uint4 *words_at(uint32_t s) const {
        return reinterpret_cast<uint4 *>(rec + (size_t)s * PF_SLOT_BYTES);
    }

    // occupancy bitmap words (at least one; tables have >= 16 slots)
    __host__ __device__ __forceinline__ uint32_t nwords() const { return (uint32_t)(((uint64_t)mask + 32) >> 5); }

    // average of component k of a cell in this table's sum format
    __device__ __forceinline__ float average(const pf_cell &c, int k) const {
        if (fsum) return float_sum_value(c.sum[k]) / (float)c.count;
        return cell_average(c.sum[k], c.count, frac_bits);
    }
};

// History of voxel values with eviction by priority, passed to kernels by value.
struct Hist {
    pf_history_slot *slot;  // word (priority byte << 56 | 56-bit key hash; all ones = empty), key, c and N
    uint32_t *stamp;        // frame last written
    uint32_t mask;
    uint32_t max_age;
};

// Fingerprint read while other lanes may claim slots: a relaxed atomic load.
__device__ __forceinline__ uint32_t load_fp_probe(uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_u64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_u32(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace pfk
