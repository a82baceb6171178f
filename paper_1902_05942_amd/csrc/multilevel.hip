// Multi-level accumulation (Section 3.3.2) for gfx950: each vertex is also
// accumulated in the voxel `levels` levels coarser that encloses its own, in
// a second table, and the lookup takes the coarser voxel's value for
// vertices whose own voxel holds fewer than a threshold of vertices.
//
// The coarser key is derived from the vertex's key alone: its level field
// grows by `levels` and each cell coordinate is floor-divided by 2^levels
// (an arithmetic shift).  For the IEEE quotients of Algorithm 1 this is the
// quantisation of the same jittered position at the coarser level, since
// floor(floor(y) / 2^k) = floor(y / 2^k) and dividing by s 2^(l'+k) scales
// the quotient by s 2^l' exactly by a power of two.  Both kernels stream
// the vertex arrays once (coalesced, one vertex per lane).
#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

__global__ __launch_bounds__(kBlock) void coarsen_kernel(const uint64_t *__restrict__ key,
                                                         const uint8_t *__restrict__ flags, uint32_t n,
                                                         uint32_t levels, uint64_t *__restrict__ key_out,
                                                         uint8_t *__restrict__ flags_out) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint8_t f = flags[i];
    if (f == PF_V_OVERFLOW) f = 0;  // its key is valid: it is accumulated at the coarser level
    uint64_t k = 0;
    if (f == 0) {
        const uint64_t K = key[i];
        const int lq = (int)((K >> 51) & 31u) - 16 + (int)levels;
        if (lq > kLevelMax) {
            f = PF_V_KEYRANGE;
        } else {
            k = ((K >> 56) << 56) | ((uint64_t)(uint32_t)(lq + 16) << 51);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int x = (int)((K >> (17 * c)) & 0x1ffffu) - 65536;
                k |= (uint64_t)(uint32_t)((x >> levels) + 65536) << (17 * c);
            }
        }
    }
    key_out[i] = k;
    flags_out[i] = f;
}

template <bool kBlend>
__global__ __launch_bounds__(kBlock) void query_multilevel_kernel(
    Tab fine, Tab coarse, const uint32_t *__restrict__ slot_f, const uint32_t *__restrict__ slot_c, const float *r,
    const float *g, const float *b, const uint8_t *__restrict__ flags_f, const uint8_t *__restrict__ flags_c,
    uint32_t n, uint32_t below, float *ro, float *go, float *bo, uint32_t *__restrict__ count_out, bool inplace) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint8_t fl = flags_f[i], flc = flags_c[i];
    const uint32_t sf = slot_f[i], sc = slot_c[i];
    if (fl != 0 || sf == kNoSlot) {  // unfiltered: the vertex's own contribution, count 0
        query_vertex<kBlend>(fine, kNoSlot, i, r, g, b, ro, go, bo, count_out, inplace);
        return;
    }
    float4 v = lookup_value(fine, sf, i, r, g, b, kBlend);
    if ((uint32_t)v.w < below && flc == 0 && sc != kNoSlot) v = lookup_value(coarse, sc, i, r, g, b, kBlend);
    ro[i] = v.x;
    go[i] = v.y;
    bo[i] = v.z;
    if (count_out) count_out[i] = (uint32_t)v.w;
}

hipError_t launch_coarsen(const uint64_t *key, const uint8_t *flags, uint32_t n, uint32_t levels, uint64_t *key_out,
                          uint8_t *flags_out, hipStream_t st) {
    const uint32_t blocks = (n + kBlock - 1) / kBlock;
    coarsen_kernel<<<blocks, kBlock, 0, st>>>(key, flags, n, levels, key_out, flags_out);
    return hipGetLastError();
}

hipError_t launch_query_multilevel(const Tab &fine, const Tab &coarse, const uint32_t *slot_f, const uint32_t *slot_c,
                                   const float *r, const float *g, const float *b, const uint8_t *flags_f,
                                   const uint8_t *flags_c, uint32_t n, uint32_t below, bool use_blend, float *ro,
                                   float *go, float *bo, uint32_t *count_out, hipStream_t st) {
    const uint32_t blocks = (n + kBlock - 1) / kBlock;
    const bool inplace = (ro == r) && (go == g) && (bo == b);
    if (use_blend)
        query_multilevel_kernel<true><<<blocks, kBlock, 0, st>>>(fine, coarse, slot_f, slot_c, r, g, b, flags_f,
                                                                 flags_c, n, below, ro, go, bo, count_out, inplace);
    else
        query_multilevel_kernel<false><<<blocks, kBlock, 0, st>>>(fine, coarse, slot_f, slot_c, r, g, b, flags_f,
                                                                  flags_c, n, below, ro, go, bo, count_out, inplace);
    return hipGetLastError();
}

}  // namespace pfk
