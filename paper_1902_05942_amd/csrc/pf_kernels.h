// Host-side launchers of the library's kernels (internal interface between
// the C ABI in pf_api.hip and the kernel translation units).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf.h"

namespace pfk {

struct Tab;

struct KeyArgs {
    float cam[3];
    float s;
    uint64_t seed;
    uint64_t idx_base;
    uint32_t mask;
};

hipError_t launch_build_keys(const float *px, const float *py, const float *pz, const float *nx, const float *ny,
                             const float *nz, const uint8_t *valid, uint32_t n, const KeyArgs &a, uint64_t *key,
                             uint32_t *fp, uint32_t *home, uint8_t *flags, hipStream_t st);

hipError_t launch_table_init(const Tab &t, hipStream_t st);
hipError_t launch_clear(const Tab &t, hipStream_t st);
hipError_t launch_insert(const Tab &t, const uint64_t *key, const float *r, const float *g, const float *b,
                         uint8_t *flags, uint32_t *slot_out, uint32_t n, uint32_t agg_width, hipStream_t st);
hipError_t launch_query(const Tab &t, const uint64_t *key, const uint32_t *slot, const float *r, const float *g,
                        const float *b, const uint8_t *flags, uint32_t n, bool use_blend, float *ro, float *go,
                        float *bo, uint32_t *count_out, hipStream_t st);
hipError_t launch_stats(const Tab &t, hipStream_t st);
hipError_t launch_temporal(const Tab &cur, const Tab *prev, float alpha_old, int mode, hipStream_t st);

}  // namespace pfk
