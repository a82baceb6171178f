// C ABI of the library (declared in include/pf.h): argument checks on the
// host, then kernel launches on the caller's stream.  No allocation, no
// synchronisation (pf_read_stats excepted).
#include <math.h>
#include <string.h>

#include "pf_device.h"
#include "pf_kernels.h"

using pfk::Tab;

namespace {

constexpr uint64_t kMaxN = 0xffffffffull;  // vertex indices are 32-bit

template <typename T>
bool aligned(const T *p) {
    return (reinterpret_cast<uintptr_t>(p) % alignof(T)) == 0;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

pf_status check_table(const pf_table *t) {
    if (!t || !t->cell || !t->key || !t->occ || !t->stats) return PF_EINVAL;
    if ((reinterpret_cast<uintptr_t>(t->cell) % 32) || !aligned(t->key) || !aligned(t->occ) ||
        !aligned(t->stats) || (t->blend && (reinterpret_cast<uintptr_t>(t->blend) % 16)))
        return PF_EINVAL;
    if (t->log2_slots < 4 || t->log2_slots > 30) return PF_ERANGE;
    if (t->max_probe < 1 || (uint64_t)t->max_probe > (1ull << t->log2_slots)) return PF_ERANGE;
    if (t->frac_bits < 8 || t->frac_bits > 40) return PF_ERANGE;
    return PF_OK;
}

Tab to_tab(const pf_table *t) {
    Tab k;
    k.cell = t->cell;
    k.key = t->key;
    k.blend = reinterpret_cast<float4 *>(t->blend);
    k.occ = t->occ;
    k.stats = reinterpret_cast<unsigned long long *>(t->stats);
    k.mask = (uint32_t)((1ull << t->log2_slots) - 1);
    k.max_probe = t->max_probe;
    k.frac_bits = t->frac_bits;
    return k;
}

pf_status launched(hipError_t e) { return e == hipSuccess ? PF_OK : PF_ELAUNCH; }

}  // namespace

extern "C" {

const char *pf_version(void) { return "pf-gfx950 1.0"; }

size_t pf_table_bytes(uint32_t log2_slots, int with_blend) {
    if (log2_slots < 4 || log2_slots > 30) return 0;
    const size_t S = (size_t)1 << log2_slots;
    size_t b = 256;                                      // alignment slack of the arena base
    b += align_up(S * sizeof(pf_cell), 256);             // cells
    b += align_up(S * sizeof(uint64_t), 256);            // keys
    b += with_blend ? align_up(S * 4 * sizeof(float), 256) : 0;
    b += align_up((S + 31) / 32 * sizeof(uint32_t), 256); // occupancy bitmap
    b += align_up(PF_STATS_LEN * sizeof(uint64_t), 256);  // statistics
    return b;
}

pf_status pf_table_carve(void *arena, uint32_t log2_slots, int with_blend, uint32_t max_probe, int32_t frac_bits,
                         pf_table *t) {
    if (!arena || !t) return PF_EINVAL;
    if (log2_slots < 4 || log2_slots > 30) return PF_ERANGE;
    if (max_probe < 1 || (uint64_t)max_probe > (1ull << log2_slots)) return PF_ERANGE;
    if (frac_bits < 8 || frac_bits > 40) return PF_ERANGE;
    const size_t S = (size_t)1 << log2_slots;
    uintptr_t p = align_up(reinterpret_cast<uintptr_t>(arena), 256);
    memset(t, 0, sizeof(*t));
    t->cell = reinterpret_cast<pf_cell *>(p);
    p += align_up(S * sizeof(pf_cell), 256);
    t->key = reinterpret_cast<uint64_t *>(p);
    p += align_up(S * sizeof(uint64_t), 256);
    if (with_blend) {
        t->blend = reinterpret_cast<float *>(p);
        p += align_up(S * 4 * sizeof(float), 256);
    }
    t->occ = reinterpret_cast<uint32_t *>(p);
    p += align_up((S + 31) / 32 * sizeof(uint32_t), 256);
    t->stats = reinterpret_cast<uint64_t *>(p);
    t->log2_slots = log2_slots;
    t->max_probe = max_probe;
    t->frac_bits = frac_bits;
    return PF_OK;
}

pf_status pf_table_init(const pf_table *t, void *stream) {
    const pf_status s = check_table(t);
    if (s != PF_OK) return s;
    return launched(pfk::launch_table_init(to_tab(t), (hipStream_t)stream));
}

pf_status pf_clear(const pf_table *t, void *stream) {
    const pf_status s = check_table(t);
    if (s != PF_OK) return s;
    return launched(pfk::launch_clear(to_tab(t), (hipStream_t)stream));
}

pf_status pf_build_keys(const float *px, const float *py, const float *pz, const float *nx, const float *ny,
                        const float *nz, const uint8_t *valid, uint64_t n, const pf_key_params *kp,
                        uint32_t log2_slots, uint64_t *key, uint32_t *fp, uint32_t *home, uint8_t *vflags,
                        void *stream) {
    if (!kp) return PF_EINVAL;
    if (n > kMaxN) return PF_EINVAL;
    if (log2_slots < 4 || log2_slots > 30) return PF_ERANGE;
    if (!(kp->s > 0.0f) || !isfinite(kp->s) || !isfinite(kp->cam[0]) || !isfinite(kp->cam[1]) ||
        !isfinite(kp->cam[2]))
        return PF_ERANGE;
    if (n == 0) return PF_OK;
    if (!px || !py || !pz || !nx || !ny || !nz || !key || !vflags) return PF_EINVAL;
    if (!aligned(px) || !aligned(py) || !aligned(pz) || !aligned(nx) || !aligned(ny) || !aligned(nz) ||
        !aligned(key) || (fp && !aligned(fp)) || (home && !aligned(home)))
        return PF_EINVAL;
    pfk::KeyArgs a;
    for (int c = 0; c < 3; ++c) a.cam[c] = kp->cam[c];
    a.s = kp->s;
    a.seed = kp->seed;
    a.idx_base = kp->idx_base;
    a.mask = (uint32_t)((1ull << log2_slots) - 1);
    return launched(pfk::launch_build_keys(px, py, pz, nx, ny, nz, valid, (uint32_t)n, a, key, fp, home, vflags,
                                           (hipStream_t)stream));
}

pf_status pf_insert_accumulate(const pf_table *t, const uint64_t *key, const float *r, const float *g,
                               const float *b, uint8_t *vflags, uint32_t *slot_out, uint64_t n, uint32_t agg_width,
                               void *stream) {
    const pf_status s = check_table(t);
    if (s != PF_OK) return s;
    if (n > kMaxN) return PF_EINVAL;
    if (agg_width > 256 || (agg_width > 1 && (agg_width & (agg_width - 1)))) return PF_ERANGE;
    if (n == 0) return PF_OK;
    if (!key || !r || !g || !b || !vflags) return PF_EINVAL;
    if (!aligned(key) || !aligned(r) || !aligned(g) || !aligned(b) || (slot_out && !aligned(slot_out)))
        return PF_EINVAL;
    return launched(pfk::launch_insert(to_tab(t), key, r, g, b, vflags, slot_out, (uint32_t)n, agg_width,
                                       (hipStream_t)stream));
}

pf_status pf_query_average(const pf_table *t, const uint64_t *key, const uint32_t *slot, const float *r_in,
                           const float *g_in, const float *b_in, const uint8_t *vflags, uint64_t n, int use_blend,
                           float *r_out, float *g_out, float *b_out, uint32_t *count_out, void *stream) {
    const pf_status s = check_table(t);
    if (s != PF_OK) return s;
    if (n > kMaxN) return PF_EINVAL;
    if (use_blend && !t->blend) return PF_EINVAL;
    if (n == 0) return PF_OK;
    if ((!key && !slot) || !r_in || !g_in || !b_in || !vflags || !r_out || !g_out || !b_out) return PF_EINVAL;
    if ((key && !aligned(key)) || (slot && !aligned(slot)) || !aligned(r_in) || !aligned(g_in) || !aligned(b_in) ||
        !aligned(r_out) || !aligned(g_out) || !aligned(b_out) || (count_out && !aligned(count_out)))
        return PF_EINVAL;
    return launched(pfk::launch_query(to_tab(t), key, slot, r_in, g_in, b_in, vflags, (uint32_t)n, use_blend != 0,
                                      r_out, g_out, b_out, count_out, (hipStream_t)stream));
}

pf_status pf_temporal_update(const pf_table *cur, const pf_table *prev, float alpha_old, int mode, void *stream) {
    pf_status s = check_table(cur);
    if (s != PF_OK) return s;
    if (!cur->blend) return PF_EINVAL;
    if (!(alpha_old >= 0.0f && alpha_old <= 1.0f)) return PF_ERANGE;
    if (mode != 0) return PF_ERANGE;
    if (prev) {
        s = check_table(prev);
        if (s != PF_OK) return s;
        if (!prev->blend) return PF_EINVAL;
        if (prev->log2_slots != cur->log2_slots) return PF_ERANGE;
    }
    Tab p;
    if (prev) p = to_tab(prev);
    return launched(pfk::launch_temporal(to_tab(cur), prev ? &p : nullptr, alpha_old, mode, (hipStream_t)stream));
}

pf_status pf_read_stats(const pf_table *t, uint64_t *host_out, void *stream) {
    const pf_status s = check_table(t);
    if (s != PF_OK) return s;
    if (!host_out) return PF_EINVAL;
    if (pfk::launch_stats(to_tab(t), (hipStream_t)stream) != hipSuccess) return PF_ELAUNCH;
    if (hipMemcpyAsync(host_out, t->stats, PF_STATS_LEN * sizeof(uint64_t), hipMemcpyDeviceToHost,
                       (hipStream_t)stream) != hipSuccess)
        return PF_ELAUNCH;
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? PF_OK : PF_ELAUNCH;
}

}  // extern "C"
