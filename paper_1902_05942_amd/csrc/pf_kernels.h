// Host-side launchers of the library's kernels (internal interface between
// the C ABI in pf_api.hip and the kernel translation units).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pf.h"

namespace pfk {

struct Tab;
struct Hist;

struct KeyArgs {
    float cam[3];
    float s;
    float inv_s;  // RN(1 / s)
    uint64_t seed;
    uint64_t idx_base;
    uint32_t mask;
};

hipError_t launch_build_keys(const float *px, const float *py, const float *pz, const float *nx, const float *ny,
                             const float *nz, const uint8_t *valid, uint32_t n, const KeyArgs &a, uint64_t *key,
                             uint32_t *fp, uint32_t *home, uint8_t *flags, hipStream_t st);

size_t binned_workspace_bytes(uint32_t n, uint32_t log2_slots);
hipError_t launch_insert_binned(const Tab &t, const uint64_t *key, const float *r, const float *g, const float *b,
                                uint8_t *flags, uint32_t *slot_out, uint32_t n, void *ws, hipStream_t st);
hipError_t launch_table_init(const Tab &t, hipStream_t st);
hipError_t launch_clear(const Tab &t, hipStream_t st);
hipError_t launch_insert(const Tab &t, const uint64_t *key, const float *r, const float *g, const float *b,
                         uint8_t *flags, uint32_t *slot_out, uint32_t n, uint32_t agg_width, hipStream_t st);
hipError_t launch_query(const Tab &t, const uint64_t *key, const uint32_t *slot, const float *r, const float *g,
                        const float *b, const uint8_t *flags, uint32_t n, bool use_blend, float *ro, float *go,
                        float *bo, uint32_t *count_out, hipStream_t st);
hipError_t launch_query_clear(const Tab &t, const uint64_t *key, const uint32_t *slot, const float *r, const float *g,
                              const float *b, const uint8_t *flags, uint32_t n, bool use_blend, float *ro, float *go,
                              float *bo, uint32_t *count_out, const Tab &clr, hipStream_t st);
hipError_t launch_stats(const Tab &t, hipStream_t st);

struct MlpArgs {
    float *w;
    uint16_t *wb;
    float *m;
    float *v;
    float *partial;
    float *loss;
    uint32_t max_batch;
};

struct GeoArgs {
    const uint64_t *key;
    const float *px, *py, *pz, *nx, *ny, *nz;
    float cam[3];
};

// A view of the batched launch as its kernel sees it: the caller's
// descriptor and the view's bucket space in the workspace.
struct ViewDev {
    pf_view d;
    uint32_t *cnt;      // [nbins * 8] records per bucket part
    uint4 *rec;         // [nbins * 8][part_cap] records of 32 bytes (two uint4)
    uint32_t nbins, part_cap;
};
size_t views_workspace_bytes(const uint64_t *n, const uint32_t *log2_slots, uint32_t nviews);
hipError_t launch_keys_insert_binned(const Tab &t, const float *px, const float *py, const float *pz,
                                     const float *nx, const float *ny, const float *nz, const uint8_t *valid,
                                     const KeyArgs &a, uint64_t *key_out, const float *r, const float *g,
                                     const float *b, uint8_t *flags, uint32_t *slot_out, uint32_t n, void *ws,
                                     hipStream_t st);
hipError_t launch_keys_insert_binned_temporal(const Tab &t, const float *px, const float *py, const float *pz,
                                              const float *nx, const float *ny, const float *nz,
                                              const uint8_t *valid, const KeyArgs &a, uint64_t *key_out,
                                              const float *r, const float *g, const float *b, uint8_t *flags,
                                              uint32_t *slot_out, uint32_t n, void *ws, const Tab *prev,
                                              float alpha_old, int mode, uint32_t cap, hipStream_t st);
bool noalloc_fits(uint32_t log2_slots);
hipError_t launch_keys_insert_binned_noalloc(const Tab &t, const float *px, const float *py, const float *pz,
                                             const float *nx, const float *ny, const float *nz,
                                             const uint8_t *valid, const KeyArgs &a, uint64_t *key_out,
                                             const float *r, const float *g, const float *b, uint8_t *flags,
                                             uint32_t *slot_out, uint32_t n, hipStream_t st);
hipError_t launch_microbench(int kind, void *buf, uint64_t bytes, uint32_t grain, uint64_t accesses, uint64_t seed,
                             uint32_t *sink, hipStream_t st);
hipError_t launch_views(const pf_view *host_views, uint32_t nviews, uint32_t block, uint32_t agg, uint32_t per_cu,
                        void *workspace, size_t workspace_bytes, hipStream_t st);
hipError_t launch_mlp_init(const MlpArgs &a, hipStream_t st);
uint32_t mlp_select_blocks(uint32_t n);
hipError_t launch_mlp_select(const uint8_t *flags, const uint32_t *count, uint32_t n, uint32_t lo, uint32_t hi,
                             uint32_t *tr_idx, uint32_t *sp_idx, uint32_t *counts, uint32_t *ws, hipStream_t st);
hipError_t launch_mlp_train(const MlpArgs &a, const Tab &t, const GeoArgs &g, const uint32_t *slot,
                            const uint32_t *train_idx, const uint32_t *counts, uint32_t batch, uint64_t seed,
                            uint32_t step, float lr, hipStream_t st);
hipError_t launch_mlp_features(const GeoArgs &g, const uint32_t *idx, uint32_t n, uint16_t *out, hipStream_t st);
hipError_t launch_mlp_infer(const MlpArgs &a, const GeoArgs &g, const uint32_t *idx, const uint32_t *counts,
                            uint32_t n_max, float *r, float *gc, float *b, hipStream_t st);
hipError_t launch_low_density(const Tab &t, uint32_t below, int mode, hipStream_t st);
hipError_t launch_history_init(const Hist &h, hipStream_t st);
hipError_t launch_resolve(const float *r, const float *g, const float *b, const float *tr, const float *tg,
                          const float *tb, const uint8_t *valid, uint32_t pixels, uint32_t verts, bool accumulate,
                          float *pr, float *pg, float *pb, hipStream_t st);
hipError_t launch_temporal_history(const Tab &cur, const Hist &h, float alpha_old, int mode, uint32_t cap,
                                   uint32_t frame, hipStream_t st);
hipError_t launch_coarsen(const uint64_t *key, const uint8_t *flags, uint32_t n, uint32_t levels, uint64_t *key_out,
                          uint8_t *flags_out, hipStream_t st);
hipError_t launch_query_multilevel(const Tab &fine, const Tab &coarse, const uint32_t *slot_f, const uint32_t *slot_c,
                                   const float *r, const float *g, const float *b, const uint8_t *flags_f,
                                   const uint8_t *flags_c, uint32_t n, uint32_t below, bool use_blend, float *ro,
                                   float *go, float *bo, uint32_t *count_out, hipStream_t st);
hipError_t launch_temporal(const Tab &cur, const Tab *prev, float alpha_old, int mode, uint32_t cap,
                           hipStream_t st);

}  // namespace pfk
