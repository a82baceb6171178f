// C ABI of the library (declared in include/pf.h): argument checks on the
// host, then kernel launches on the caller's stream.  No allocation, no
// synchronisation (pf_read_stats excepted).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "pf_device.h"
#include "pf_kernels.h"

using pfk::Tab;

namespace {

constexpr uint64_t kMaxN = PF_MAX_VERTICES;  // 32-bit indices: n + block - 1 cannot wrap

template <typename T>
bool aligned(const T *p) {
    return (reinterpret_cast<uintptr_t>(p) % alignof(T)) == 0;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

pf_status check_table(const pf_table *t) {
    if (!t || !t->cell || !t->key || !t->occ || !t->stats) return PF_EINVAL;
    const char *base = reinterpret_cast<const char *>(t->cell);
    if ((reinterpret_cast<uintptr_t>(t->cell) % PF_SLOT_BYTES) || reinterpret_cast<const char *>(t->key) != base + 32 ||
        (t->blend && reinterpret_cast<const char *>(t->blend) != base + 48) || !aligned(t->occ) || !aligned(t->stats))
        return PF_EINVAL;
    if (t->log2_slots < 4 || t->log2_slots > 30) return PF_ERANGE;
    if (t->max_probe < 1 || (uint64_t)t->max_probe > (1ull << t->log2_slots)) return PF_ERANGE;
    if (t->frac_bits < 8 || t->frac_bits > 40) return PF_ERANGE;
    if (t->sum_format != PF_SUMS_FIXED64 && t->sum_format != PF_SUMS_FLOAT32) return PF_EINVAL;
    return PF_OK;
}

Tab to_tab(const pf_table *t) {
    Tab k;
    k.rec = reinterpret_cast<unsigned char *>(t->cell);
    k.occ = t->occ;
    k.stats = reinterpret_cast<unsigned long long *>(t->stats);
    k.mask = (uint32_t)((1ull << t->log2_slots) - 1);
    k.max_probe = t->max_probe;
    k.frac_bits = t->frac_bits;
    k.fsum = t->sum_format == PF_SUMS_FLOAT32 ? 1u : 0u;
    return k;
}

pf_status launched(hipError_t e) { return e == hipSuccess ? PF_OK : PF_ELAUNCH; }

}  // namespace

extern "C" {

const char *pf_version(void) { return "pf-gfx950 1.0"; }

uint64_t pf_wall_clock_hz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) return 0;
    return (uint64_t)khz * 1000ull;
}

size_t pf_table_bytes(uint32_t log2_slots, int with_blend) {
    if (log2_slots < 4 || log2_slots > 30) return 0;
    const size_t S = (size_t)1 << log2_slots;
    size_t b = 256;                                      // alignment slack of the arena base
    b += align_up(S * PF_SLOT_BYTES, 256);               // slot records: cell, key, temporal value
    (void)with_blend;                                    // the records always keep the value's space
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
    t->key = reinterpret_cast<uint64_t *>(p + 32);
    t->blend = with_blend ? reinterpret_cast<float *>(p + 48) : nullptr;
    p += align_up(S * PF_SLOT_BYTES, 256);
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
    a.inv_s = 1.0f / kp->s;
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

size_t pf_insert_workspace_bytes(uint64_t n, uint32_t log2_slots) {
    if (n > kMaxN || log2_slots < 4) return 0;
    return pfk::binned_workspace_bytes((uint32_t)n, log2_slots);
}

pf_status pf_insert_accumulate_binned(const pf_table *t, const uint64_t *key, const float *r, const float *g,
                                      const float *b, uint8_t *vflags, uint32_t *slot_out, uint64_t n,
                                      void *workspace, size_t workspace_bytes, void *stream) {
    const pf_status s = check_table(t);
    if (s != PF_OK) return s;
    if (n > kMaxN) return PF_EINVAL;
    if (t->sum_format != PF_SUMS_FIXED64) return PF_EINVAL;
    const size_t need = pf_insert_workspace_bytes(n, t->log2_slots);
    if (need == 0) return PF_ERANGE;
    if (n == 0) return PF_OK;
    if (!key || !r || !g || !b || !vflags || !slot_out || !workspace || workspace_bytes < need) return PF_EINVAL;
    if (!aligned(key) || !aligned(r) || !aligned(g) || !aligned(b) || !aligned(slot_out)) return PF_EINVAL;
    return launched(pfk::launch_insert_binned(to_tab(t), key, r, g, b, vflags, slot_out, (uint32_t)n, workspace,
                                              (hipStream_t)stream));
}

// workspace_bytes of check_keys_insert for a call without a workspace
constexpr size_t kNoWorkspace = ~(size_t)0;

// The checks of pf_build_keys_insert_binned; fills a.  PF_OK with *empty
// set when n == 0 (nothing to launch).
static pf_status check_keys_insert(const pf_table *t, const float *px, const float *py, const float *pz,
                                   const float *nx, const float *ny, const float *nz, const pf_key_params *kp,
                                   const float *r, const float *g, const float *b, uint64_t n, const uint64_t *key,
                                   const uint8_t *vflags, const uint32_t *slot_out, const void *workspace,
                                   size_t workspace_bytes, pfk::KeyArgs &a, bool &empty) {
    const pf_status s = check_table(t);
    if (s != PF_OK) return s;
    if (!kp) return PF_EINVAL;
    if (n > kMaxN) return PF_EINVAL;
    if (t->sum_format != PF_SUMS_FIXED64) return PF_EINVAL;
    if (!(kp->s > 0.0f) || !isfinite(kp->s) || !isfinite(kp->cam[0]) || !isfinite(kp->cam[1]) ||
        !isfinite(kp->cam[2]))
        return PF_ERANGE;
    // no_workspace: the no-allocation variant, whose workspace is the
    // library's own scratch (checked by the caller)
    const bool no_workspace = workspace == nullptr && workspace_bytes == kNoWorkspace;
    const size_t need = pf_insert_workspace_bytes(n, t->log2_slots);
    if (need == 0) return PF_ERANGE;
    empty = n == 0;
    if (empty) return PF_OK;
    if (!px || !py || !pz || !nx || !ny || !nz || !r || !g || !b || !vflags || !slot_out)
        return PF_EINVAL;
    if (!no_workspace && (!workspace || workspace_bytes < need)) return PF_EINVAL;
    if (!aligned(px) || !aligned(py) || !aligned(pz) || !aligned(nx) || !aligned(ny) || !aligned(nz) ||
        !aligned(r) || !aligned(g) || !aligned(b) || !aligned(slot_out) || (key && !aligned(key)))
        return PF_EINVAL;
    for (int c = 0; c < 3; ++c) a.cam[c] = kp->cam[c];
    a.s = kp->s;
    a.inv_s = 1.0f / kp->s;
    a.seed = kp->seed;
    a.idx_base = kp->idx_base;
    a.mask = (uint32_t)((1ull << t->log2_slots) - 1);
    return PF_OK;
}

pf_status pf_build_keys_insert_binned(const pf_table *t, const float *px, const float *py, const float *pz,
                                      const float *nx, const float *ny, const float *nz, const uint8_t *valid,
                                      const pf_key_params *kp, const float *r, const float *g, const float *b,
                                      uint64_t n, uint64_t *key, uint8_t *vflags, uint32_t *slot_out,
                                      void *workspace, size_t workspace_bytes, void *stream) {
    pfk::KeyArgs a;
    bool empty = false;
    const pf_status s = check_keys_insert(t, px, py, pz, nx, ny, nz, kp, r, g, b, n, key, vflags, slot_out, workspace,
                                          workspace_bytes, a, empty);
    if (s != PF_OK || empty) return s;
    return launched(pfk::launch_keys_insert_binned(to_tab(t), px, py, pz, nx, ny, nz, valid, a, key, r, g, b, vflags,
                                                   slot_out, (uint32_t)n, workspace, (hipStream_t)stream));
}

pf_status pf_build_keys_insert_binned_noalloc(const pf_table *t, const float *px, const float *py, const float *pz,
                                              const float *nx, const float *ny, const float *nz, const uint8_t *valid,
                                              const pf_key_params *kp, const float *r, const float *g, const float *b,
                                              uint64_t n, uint64_t *key, uint8_t *vflags, uint32_t *slot_out,
                                              void *stream) {
    pfk::KeyArgs a;
    bool empty = false;
    const pf_status s = check_keys_insert(t, px, py, pz, nx, ny, nz, kp, r, g, b, n, key, vflags, slot_out, nullptr,
                                          kNoWorkspace, a, empty);
    if (s != PF_OK) return s;
    if (!pfk::noalloc_fits(t->log2_slots)) return PF_ERANGE;
    if (empty) return PF_OK;
    return launched(pfk::launch_keys_insert_binned_noalloc(to_tab(t), px, py, pz, nx, ny, nz, valid, a, key, r, g, b,
                                                           vflags, slot_out, (uint32_t)n, (hipStream_t)stream));
}

pf_status pf_build_keys_insert_binned_temporal(const pf_table *t, const float *px, const float *py, const float *pz,
                                               const float *nx, const float *ny, const float *nz,
                                               const uint8_t *valid, const pf_key_params *kp, const float *r,
                                               const float *g, const float *b, uint64_t n, uint64_t *key,
                                               uint8_t *vflags, uint32_t *slot_out, void *workspace,
                                               size_t workspace_bytes, const pf_table *prev, float alpha_old,
                                               uint32_t max_samples, void *stream) {
    pfk::KeyArgs a;
    bool empty = false;
    pf_status s = check_keys_insert(t, px, py, pz, nx, ny, nz, kp, r, g, b, n, key, vflags, slot_out, workspace,
                                    workspace_bytes, a, empty);
    if (s != PF_OK) return s;
    if (!t->blend) return PF_EINVAL;
    if (prev) {
        s = check_table(prev);
        if (s != PF_OK) return s;
        if (!prev->blend) return PF_EINVAL;
        if (prev->log2_slots != t->log2_slots) return PF_ERANGE;
        if (prev->cell == t->cell) return PF_EINVAL;
    }
    if (max_samples > PF_MAX_SAMPLES) return PF_ERANGE;
    if (max_samples == 0 && !(alpha_old >= 0.0f && alpha_old <= 1.0f)) return PF_ERANGE;
    if (empty) return PF_OK;
    pfk::Tab p;
    if (prev) p = to_tab(prev);
    return launched(pfk::launch_keys_insert_binned_temporal(
        to_tab(t), px, py, pz, nx, ny, nz, valid, a, key, r, g, b, vflags, slot_out, (uint32_t)n, workspace,
        prev ? &p : nullptr, alpha_old, max_samples ? 1 : 0, max_samples ? max_samples : PF_MAX_SAMPLES,
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

pf_status pf_query_average_clear(const pf_table *t, const uint64_t *key, const uint32_t *slot, const float *r_in,
                                 const float *g_in, const float *b_in, const uint8_t *vflags, uint64_t n,
                                 int use_blend, float *r_out, float *g_out, float *b_out, uint32_t *count_out,
                                 const pf_table *clear, void *stream) {
    pf_status s = check_table(t);
    if (s != PF_OK) return s;
    if (!clear) return PF_EINVAL;
    s = check_table(clear);
    if (s != PF_OK) return s;
    {  // the two tables' slot records must not overlap
        const uintptr_t a0 = (uintptr_t)t->cell, a1 = a0 + ((uintptr_t)PF_SLOT_BYTES << t->log2_slots);
        const uintptr_t c0 = (uintptr_t)clear->cell, c1 = c0 + ((uintptr_t)PF_SLOT_BYTES << clear->log2_slots);
        if (a0 < c1 && c0 < a1) return PF_EINVAL;
    }
    if (n > kMaxN) return PF_EINVAL;
    if (use_blend && !t->blend) return PF_EINVAL;
    if (n == 0) return launched(pfk::launch_clear(to_tab(clear), (hipStream_t)stream));
    if ((!key && !slot) || !r_in || !g_in || !b_in || !vflags || !r_out || !g_out || !b_out) return PF_EINVAL;
    if ((key && !aligned(key)) || (slot && !aligned(slot)) || !aligned(r_in) || !aligned(g_in) || !aligned(b_in) ||
        !aligned(r_out) || !aligned(g_out) || !aligned(b_out) || (count_out && !aligned(count_out)))
        return PF_EINVAL;
    return launched(pfk::launch_query_clear(to_tab(t), key, slot, r_in, g_in, b_in, vflags, (uint32_t)n,
                                            use_blend != 0, r_out, g_out, b_out, count_out, to_tab(clear),
                                            (hipStream_t)stream));
}

static pf_status temporal(const pf_table *cur, const pf_table *prev, float alpha_old, int mode, uint32_t cap,
                          void *stream) {
    pf_status s = check_table(cur);
    if (s != PF_OK) return s;
    if (!cur->blend) return PF_EINVAL;
    if (prev) {
        s = check_table(prev);
        if (s != PF_OK) return s;
        if (!prev->blend) return PF_EINVAL;
        if (prev->log2_slots != cur->log2_slots) return PF_ERANGE;
    }
    Tab p;
    if (prev) p = to_tab(prev);
    return launched(pfk::launch_temporal(to_tab(cur), prev ? &p : nullptr, alpha_old, mode, cap, (hipStream_t)stream));
}

pf_status pf_temporal_update(const pf_table *cur, const pf_table *prev, float alpha_old, int mode, void *stream) {
    const int base = mode & ~PF_TEMPORAL_ACROSS_LEVELS;
    if (base == 0 && !(alpha_old >= 0.0f && alpha_old <= 1.0f)) return PF_ERANGE;
    if (base != 0 && base != 1) return PF_ERANGE;
    return temporal(cur, prev, alpha_old, mode, PF_MAX_SAMPLES, stream);
}

pf_status pf_temporal_integrate(const pf_table *cur, const pf_table *prev, uint32_t max_samples, void *stream) {
    if (max_samples < 1 || max_samples > PF_MAX_SAMPLES) return PF_ERANGE;
    return temporal(cur, prev, 0.0f, 1, max_samples, stream);
}

size_t pf_history_bytes(uint32_t log2_slots) {
    if (log2_slots < 4 || log2_slots > 30) return 0;
    const size_t S = (size_t)1 << log2_slots;
    return 256 + align_up(S * sizeof(pf_history_slot), 256) + align_up(S * sizeof(uint32_t), 256);
}

pf_status pf_history_carve(void *arena, uint32_t log2_slots, uint32_t max_age, pf_history *h) {
    if (!arena || !h) return PF_EINVAL;
    if (log2_slots < 4 || log2_slots > 30) return PF_ERANGE;
    const size_t S = (size_t)1 << log2_slots;
    uintptr_t p = align_up(reinterpret_cast<uintptr_t>(arena), 256);
    h->slot = reinterpret_cast<pf_history_slot *>(p);
    p += align_up(S * sizeof(pf_history_slot), 256);
    h->stamp = reinterpret_cast<uint32_t *>(p);
    h->log2_slots = log2_slots;
    h->max_age = max_age;
    return PF_OK;
}

static bool history_ok(const pf_history *h) {
    return h && h->slot && h->stamp && (reinterpret_cast<uintptr_t>(h->slot) % 32) == 0 && aligned(h->stamp) &&
           h->log2_slots >= 4 && h->log2_slots <= 30;
}

static pfk::Hist to_hist(const pf_history *h) {
    pfk::Hist d;
    d.slot = h->slot;
    d.stamp = h->stamp;
    d.mask = (uint32_t)((1ull << h->log2_slots) - 1);
    d.max_age = h->max_age;
    return d;
}

pf_status pf_history_init(const pf_history *h, void *stream) {
    if (!history_ok(h)) return PF_EINVAL;
    return launched(pfk::launch_history_init(to_hist(h), (hipStream_t)stream));
}

pf_status pf_temporal_history(const pf_table *cur, const pf_history *h, float alpha_old, int mode,
                              uint32_t max_samples, uint32_t frame, void *stream) {
    const pf_status s = check_table(cur);
    if (s != PF_OK) return s;
    if (!cur->blend || !history_ok(h)) return PF_EINVAL;
    if (mode != 0 && mode != 1) return PF_ERANGE;
    if (mode == 0 && !(alpha_old >= 0.0f && alpha_old <= 1.0f)) return PF_ERANGE;
    if (mode == 1 && (max_samples < 1 || max_samples > PF_MAX_SAMPLES)) return PF_ERANGE;
    return launched(pfk::launch_temporal_history(to_tab(cur), to_hist(h), alpha_old, mode,
                                                 mode == 1 ? max_samples : PF_MAX_SAMPLES, frame,
                                                 (hipStream_t)stream));
}

pf_status pf_resolve_pixels(const float *r, const float *g, const float *b, const float *tr, const float *tg,
                            const float *tb, const uint8_t *valid, uint64_t pixels, uint32_t verts_per_path,
                            int accumulate, float *pr, float *pg, float *pb, void *stream) {
    if (verts_per_path && pixels > kMaxN / verts_per_path) return PF_EINVAL;
    if (pixels == 0) return PF_OK;
    if (!r || !g || !b || !pr || !pg || !pb || !aligned(r) || !aligned(g) || !aligned(b) || !aligned(pr) ||
        !aligned(pg) || !aligned(pb))
        return PF_EINVAL;
    const int nt = (tr != nullptr) + (tg != nullptr) + (tb != nullptr);
    if (nt != 0 && nt != 3) return PF_EINVAL;
    if (nt == 3 && (!aligned(tr) || !aligned(tg) || !aligned(tb))) return PF_EINVAL;
    return launched(pfk::launch_resolve(r, g, b, tr, tg, tb, valid, (uint32_t)pixels, verts_per_path,
                                        accumulate != 0, pr, pg, pb, (hipStream_t)stream));
}

pf_status pf_low_density_fallback(const pf_table *t, uint32_t below, int mode, void *stream) {
    pf_status s = check_table(t);
    if (s != PF_OK) return s;
    if (!t->blend || t->sum_format != PF_SUMS_FIXED64) return PF_EINVAL;
    if (mode != PF_LD_NEIGHBOURS && mode != PF_LD_NORMALS) return PF_ERANGE;
    if (below <= 1) return PF_OK;
    return launched(pfk::launch_low_density(to_tab(t), below, mode, (hipStream_t)stream));
}

pf_status pf_coarsen_keys(const uint64_t *key, const uint8_t *vflags, uint64_t n, uint32_t levels,
                          uint64_t *key_out, uint8_t *vflags_out, void *stream) {
    if (n > kMaxN) return PF_EINVAL;
    if (levels < 1 || levels > 31) return PF_ERANGE;
    if (n == 0) return PF_OK;
    if (!key || !vflags || !key_out || !vflags_out || !aligned(key) || !aligned(key_out)) return PF_EINVAL;
    return launched(pfk::launch_coarsen(key, vflags, (uint32_t)n, levels, key_out, vflags_out, (hipStream_t)stream));
}

pf_status pf_query_multilevel(const pf_table *fine, const pf_table *coarse, const uint32_t *slot,
                              const uint32_t *slot_coarse, const float *r_in, const float *g_in,
                              const float *b_in, const uint8_t *vflags, const uint8_t *vflags_coarse,
                              uint64_t n, uint32_t below, int use_blend, float *r_out, float *g_out,
                              float *b_out, uint32_t *count_out, void *stream) {
    pf_status s = check_table(fine);
    if (s != PF_OK) return s;
    s = check_table(coarse);
    if (s != PF_OK) return s;
    if (n > kMaxN) return PF_EINVAL;
    if (use_blend && (!fine->blend || !coarse->blend)) return PF_EINVAL;
    if (n == 0) return PF_OK;
    if (!slot || !slot_coarse || !r_in || !g_in || !b_in || !vflags || !vflags_coarse || !r_out || !g_out ||
        !b_out)
        return PF_EINVAL;
    if (!aligned(slot) || !aligned(slot_coarse) || !aligned(r_in) || !aligned(g_in) || !aligned(b_in) ||
        !aligned(r_out) || !aligned(g_out) || !aligned(b_out) || (count_out && !aligned(count_out)))
        return PF_EINVAL;
    return launched(pfk::launch_query_multilevel(to_tab(fine), to_tab(coarse), slot, slot_coarse, r_in, g_in, b_in,
                                                 vflags, vflags_coarse, (uint32_t)n, below, use_blend != 0, r_out,
                                                 g_out, b_out, count_out, (hipStream_t)stream));
}

// ------------------------------------------------------------------ learned fallback
namespace {
size_t mlp_partial_floats(uint32_t max_batch) { return (size_t)(max_batch / PF_MLP_BLOCK_SAMPLES) * (PF_MLP_NPARAM + 1); }

bool mlp_ok(const pf_mlp *m) {
    return m && m->w && m->wb && m->m && m->v && m->partial && m->loss && m->max_batch &&
           m->max_batch % PF_MLP_BLOCK_SAMPLES == 0 && aligned(m->w) && reinterpret_cast<uintptr_t>(m->wb) % 16 == 0 &&
           aligned(m->m) &&
           aligned(m->v) && aligned(m->partial) && aligned(m->loss);
}

pfk::MlpArgs to_mlp(const pf_mlp *m) {
    pfk::MlpArgs a;
    a.w = m->w;
    a.wb = m->wb;
    a.m = m->m;
    a.v = m->v;
    a.partial = m->partial;
    a.loss = m->loss;
    a.max_batch = m->max_batch;
    return a;
}

bool geo_ok(const pf_geometry *g) {
    return g && g->key && g->px && g->py && g->pz && g->nx && g->ny && g->nz && aligned(g->key) && aligned(g->px) &&
           aligned(g->py) && aligned(g->pz) && aligned(g->nx) && aligned(g->ny) && aligned(g->nz) &&
           isfinite(g->cam[0]) && isfinite(g->cam[1]) && isfinite(g->cam[2]);
}

pfk::GeoArgs to_geo(const pf_geometry *g) {
    pfk::GeoArgs a;
    a.key = g->key;
    a.px = g->px;
    a.py = g->py;
    a.pz = g->pz;
    a.nx = g->nx;
    a.ny = g->ny;
    a.nz = g->nz;
    for (int c = 0; c < 3; ++c) a.cam[c] = g->cam[c];
    return a;
}
}  // namespace

size_t pf_mlp_bytes(uint32_t max_batch) {
    if (max_batch == 0 || max_batch % PF_MLP_BLOCK_SAMPLES || max_batch > (1u << 20)) return 0;
    size_t b = 256;
    b += align_up(PF_MLP_NPARAM * sizeof(float), 256) * 3;   // w, m, v
    b += align_up(PF_MLP_NPARAM * sizeof(uint16_t), 256);    // wb
    b += align_up(mlp_partial_floats(max_batch) * sizeof(float), 256);
    b += 256;                                                // loss
    return b;
}

pf_status pf_mlp_carve(void *arena, uint32_t max_batch, pf_mlp *m) {
    if (!arena || !m) return PF_EINVAL;
    if (pf_mlp_bytes(max_batch) == 0) return PF_ERANGE;
    uintptr_t p = align_up(reinterpret_cast<uintptr_t>(arena), 256);
    memset(m, 0, sizeof(*m));
    m->w = reinterpret_cast<float *>(p);
    p += align_up(PF_MLP_NPARAM * sizeof(float), 256);
    m->m = reinterpret_cast<float *>(p);
    p += align_up(PF_MLP_NPARAM * sizeof(float), 256);
    m->v = reinterpret_cast<float *>(p);
    p += align_up(PF_MLP_NPARAM * sizeof(float), 256);
    m->wb = reinterpret_cast<uint16_t *>(p);
    p += align_up(PF_MLP_NPARAM * sizeof(uint16_t), 256);
    m->partial = reinterpret_cast<float *>(p);
    p += align_up(mlp_partial_floats(max_batch) * sizeof(float), 256);
    m->loss = reinterpret_cast<float *>(p);
    m->max_batch = max_batch;
    return PF_OK;
}

pf_status pf_mlp_init(const pf_mlp *m, void *stream) {
    if (!mlp_ok(m)) return PF_EINVAL;
    return launched(pfk::launch_mlp_init(to_mlp(m), (hipStream_t)stream));
}

size_t pf_mlp_select_workspace_bytes(uint64_t n) {
    if (n > kMaxN) return 0;
    // two counts per block of 4096 vertices, then a mask word per 16 vertices
    const size_t blocks = pfk::mlp_select_blocks((uint32_t)n);
    return (2 * blocks + blocks * 256) * sizeof(uint32_t) + 4;
}

pf_status pf_mlp_select(const uint8_t *vflags, const uint32_t *count, uint64_t n, uint32_t sparse_below,
                        uint32_t train_from, uint32_t *train_idx, uint32_t *sparse_idx, uint32_t *counts,
                        void *workspace, void *stream) {
    if (n > kMaxN) return PF_EINVAL;
    if (!counts || !aligned(counts)) return PF_EINVAL;
    if (n > 0 && (!vflags || !count || !train_idx || !sparse_idx || !workspace)) return PF_EINVAL;
    if ((count && !aligned(count)) || (train_idx && !aligned(train_idx)) || (sparse_idx && !aligned(sparse_idx)) ||
        (workspace && !aligned(reinterpret_cast<uint32_t *>(workspace))))
        return PF_EINVAL;
    return launched(pfk::launch_mlp_select(vflags, count, (uint32_t)n, sparse_below, train_from, train_idx,
                                           sparse_idx, counts, reinterpret_cast<uint32_t *>(workspace),
                                           (hipStream_t)stream));
}

pf_status pf_mlp_train_step(const pf_mlp *m, const pf_table *t, const pf_geometry *g, const uint32_t *slot,
                            const uint32_t *train_idx, const uint32_t *counts, uint32_t batch, uint64_t seed,
                            uint32_t step, float lr, void *stream) {
    if (!mlp_ok(m)) return PF_EINVAL;
    pf_status s = check_table(t);
    if (s != PF_OK) return s;
    if (!geo_ok(g) || !slot || !train_idx || !counts || !aligned(slot) || !aligned(train_idx) || !aligned(counts))
        return PF_EINVAL;
    if (batch == 0 || batch % PF_MLP_BLOCK_SAMPLES || batch > m->max_batch) return PF_ERANGE;
    if (step == 0 || !(lr > 0.0f) || !isfinite(lr)) return PF_ERANGE;
    return launched(pfk::launch_mlp_train(to_mlp(m), to_tab(t), to_geo(g), slot, train_idx, counts, batch, seed,
                                          step, lr, (hipStream_t)stream));
}

pf_status pf_mlp_features(const pf_geometry *g, const uint32_t *idx, uint64_t n, uint16_t *out, void *stream) {
    if (n > kMaxN / PF_MLP_IN) return PF_ERANGE;
    if (n == 0) return PF_OK;
    if (!geo_ok(g) || !idx || !out || !aligned(idx) || !aligned(out)) return PF_EINVAL;
    return launched(pfk::launch_mlp_features(to_geo(g), idx, (uint32_t)n, out, (hipStream_t)stream));
}

pf_status pf_mlp_infer(const pf_mlp *m, const pf_geometry *g, const uint32_t *sparse_idx, const uint32_t *counts,
                       uint64_t n_max, float *r, float *gch, float *b, void *stream) {
    if (!mlp_ok(m)) return PF_EINVAL;
    if (n_max > kMaxN) return PF_ERANGE;
    if (!geo_ok(g) || !sparse_idx || !counts || !r || !gch || !b || !aligned(sparse_idx) || !aligned(counts) ||
        !aligned(r) || !aligned(gch) || !aligned(b))
        return PF_EINVAL;
    if (n_max == 0) return PF_OK;
    return launched(pfk::launch_mlp_infer(to_mlp(m), to_geo(g), sparse_idx, counts, (uint32_t)n_max, r, gch, b,
                                          (hipStream_t)stream));
}

// ------------------------------------------------------------------ many views
static_assert(sizeof(pf_view) == 296, "pf_view layout is part of the ABI");
static_assert(sizeof(pf_table) == 56, "pf_table layout is part of the ABI");

size_t pf_views_workspace_bytes(const uint64_t *n, const uint32_t *log2_slots, uint32_t nviews) {
    if (!n || !log2_slots || nviews == 0 || nviews > PF_MAX_VIEWS) return 0;
    for (uint32_t v = 0; v < nviews; ++v)
        if (n[v] > kMaxN || log2_slots[v] < 4 || log2_slots[v] > 30) return 0;
    return pfk::views_workspace_bytes(n, log2_slots, nviews);
}

namespace {
pf_status check_view(const pf_view &d) {
    if (!d.px || !d.py || !d.pz || !d.nx || !d.ny || !d.nz || !d.r || !d.g || !d.b || !d.vflags || !d.slot ||
        !d.r_out || !d.g_out || !d.b_out)
        return PF_EINVAL;
    if (!aligned(d.px) || !aligned(d.py) || !aligned(d.pz) || !aligned(d.nx) || !aligned(d.ny) || !aligned(d.nz) ||
        !aligned(d.r) || !aligned(d.g) || !aligned(d.b) || (d.key && !aligned(d.key)) || !aligned(d.slot) ||
        !aligned(d.r_out) || !aligned(d.g_out) || !aligned(d.b_out) || (d.count_out && !aligned(d.count_out)))
        return PF_EINVAL;
    if (d.r_out == d.r || d.g_out == d.g || d.b_out == d.b) return PF_EINVAL;
    if (d.n > kMaxN) return PF_EINVAL;
    pf_status s = check_table(&d.cur);
    if (s != PF_OK) return s;
    if (d.cur.sum_format != PF_SUMS_FIXED64) return PF_EINVAL;
    if (d.temporal && !d.cur.blend) return PF_EINVAL;
    if (d.prev.cell) {
        s = check_table(&d.prev);
        if (s != PF_OK) return s;
        if (!d.prev.blend || d.prev.log2_slots != d.cur.log2_slots || d.prev.cell == d.cur.cell) return PF_EINVAL;
    }
    if (!(d.kp.s > 0.0f) || !isfinite(d.kp.s) || !isfinite(d.kp.cam[0]) || !isfinite(d.kp.cam[1]) ||
        !isfinite(d.kp.cam[2]))
        return PF_ERANGE;
    if (!(d.alpha_old >= 0.0f && d.alpha_old <= 1.0f)) return PF_ERANGE;
    return PF_OK;
}
}  // namespace

size_t pf_views_concurrent_workspace_bytes(const uint64_t *n, const uint32_t *log2_slots, uint32_t nviews) {
    if (!n || !log2_slots || nviews == 0 || nviews > PF_MAX_VIEWS) return 0;
    size_t total = 0;
    for (uint32_t v = 0; v < nviews; ++v) {
        if (n[v] > kMaxN || log2_slots[v] < 4 || log2_slots[v] > 30) return 0;
        const size_t b = pf_insert_workspace_bytes(n[v], log2_slots[v]);
        if (b == 0) return 0;
        total += align_up(b, 256);
    }
    return total;
}

namespace {
// Library streams of a device for pf_filter_views_concurrent (default
// priority, non-blocking), with the events of one fork and join; created at
// the first call on the device.  `lock` serialises the calls' host side,
// which records and waits on the shared events.
constexpr int kViewStreams = 4;
struct ViewStreams {
    std::mutex lock;
    bool ready = false;
    hipStream_t s[kViewStreams];
    hipEvent_t fork, join[kViewStreams];
};
ViewStreams g_view_streams[64];

hipError_t view_streams(int dev, ViewStreams *&vs) {
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    vs = &g_view_streams[dev];
    if (vs->ready) return hipSuccess;
    hipError_t e = hipEventCreateWithFlags(&vs->fork, hipEventDisableTiming);
    for (int k = 0; k < kViewStreams && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&vs->s[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&vs->join[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) vs->ready = true;
    return e;
}
}  // namespace

pf_status pf_filter_views_concurrent(const pf_view *views, uint32_t nviews, uint32_t nstreams, void *workspace,
                                     size_t workspace_bytes, void *stream) {
    if (!views || !workspace || (reinterpret_cast<uintptr_t>(workspace) % 256)) return PF_EINVAL;
    if (nviews == 0 || nviews > PF_MAX_VIEWS || nstreams == 0 || nstreams > (uint32_t)kViewStreams) return PF_ERANGE;
    uint64_t n[PF_MAX_VIEWS];
    uint32_t lg[PF_MAX_VIEWS];
    for (uint32_t v = 0; v < nviews; ++v) {
        const pf_view &d = views[v];
        const pf_status s = check_view(d);
        if (s != PF_OK) return s;
        if (!(d.kp.s > 0.0f) || !isfinite(d.kp.s) || !isfinite(d.kp.cam[0]) || !isfinite(d.kp.cam[1]) ||
            !isfinite(d.kp.cam[2]))
            return PF_ERANGE;
        if (d.temporal && !(d.alpha_old >= 0.0f && d.alpha_old <= 1.0f)) return PF_ERANGE;
        for (uint32_t u = 0; u < v; ++u)  // every view owns its tables
            if (views[u].cur.cell == d.cur.cell || views[u].cur.cell == d.prev.cell ||
                views[u].prev.cell == d.cur.cell)
                return PF_EINVAL;
        n[v] = d.n;
        lg[v] = d.cur.log2_slots;
    }
    if (workspace_bytes < pf_views_concurrent_workspace_bytes(n, lg, nviews)) return PF_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PF_ELAUNCH;
    ViewStreams *vs = nullptr;
    static std::mutex create;
    {
        std::lock_guard<std::mutex> g(create);
        if (view_streams(dev, vs) != hipSuccess) return PF_ELAUNCH;
    }
    std::lock_guard<std::mutex> g(vs->lock);
    hipStream_t caller = (hipStream_t)stream;
    if (hipEventRecord(vs->fork, caller) != hipSuccess) return PF_ELAUNCH;
    const int K = (int)nstreams;
    for (int k = 0; k < K; ++k)
        if (hipStreamWaitEvent(vs->s[k], vs->fork, 0) != hipSuccess) return PF_ELAUNCH;
    // largest views first, each to the stream with the fewest vertices so far
    uint32_t order[PF_MAX_VIEWS];
    for (uint32_t v = 0; v < nviews; ++v) order[v] = v;
    std::sort(order, order + nviews, [&](uint32_t a, uint32_t b) { return n[a] > n[b] || (n[a] == n[b] && a < b); });
    uint64_t load[kViewStreams] = {};
    size_t off[PF_MAX_VIEWS];
    size_t o = 0;
    for (uint32_t v = 0; v < nviews; ++v) {
        off[v] = o;
        o += align_up(pf_insert_workspace_bytes(n[v], lg[v]), 256);
    }
    pf_status status = PF_OK;
    for (uint32_t i = 0; i < nviews && status == PF_OK; ++i) {
        const uint32_t v = order[i];
        int k = 0;
        for (int j = 1; j < K; ++j)
            if (load[j] < load[k]) k = j;
        load[k] += n[v] + 1;
        const pf_view &d = views[v];
        void *st = vs->s[k];
        void *ws = reinterpret_cast<char *>(workspace) + off[v];
        const size_t wsb = pf_insert_workspace_bytes(n[v], lg[v]);
        const pf_table *prev = d.prev.cell ? &d.prev : nullptr;
        status = pf_clear(&d.cur, st);
        if (status == PF_OK)
            status = d.temporal
                         ? pf_build_keys_insert_binned_temporal(&d.cur, d.px, d.py, d.pz, d.nx, d.ny, d.nz, d.valid,
                                                                &d.kp, d.r, d.g, d.b, d.n, d.key, d.vflags, d.slot, ws,
                                                                wsb, prev, d.alpha_old, 0, st)
                         : pf_build_keys_insert_binned(&d.cur, d.px, d.py, d.pz, d.nx, d.ny, d.nz, d.valid, &d.kp,
                                                       d.r, d.g, d.b, d.n, d.key, d.vflags, d.slot, ws, wsb, st);
        if (status == PF_OK)
            status = prev ? pf_query_average_clear(&d.cur, nullptr, d.slot, d.r, d.g, d.b, d.vflags, d.n, d.temporal,
                                                   d.r_out, d.g_out, d.b_out, d.count_out, prev, st)
                          : pf_query_average(&d.cur, nullptr, d.slot, d.r, d.g, d.b, d.vflags, d.n, d.temporal,
                                             d.r_out, d.g_out, d.b_out, d.count_out, st);
    }
    // join every stream back into the caller's, also after a failure
    for (int k = 0; k < K; ++k)
        if (hipEventRecord(vs->join[k], vs->s[k]) != hipSuccess ||
            hipStreamWaitEvent(caller, vs->join[k], 0) != hipSuccess)
            status = PF_ELAUNCH;
    return status;
}

pf_status pf_filter_views(const pf_view *views, uint32_t nviews, uint32_t block, uint32_t agg_width,
                          uint32_t grid_per_cu, void *workspace, size_t workspace_bytes, void *stream) {
    if (!views || !workspace || (reinterpret_cast<uintptr_t>(workspace) % 256)) return PF_EINVAL;
    if (nviews == 0 || nviews > PF_MAX_VIEWS) return PF_ERANGE;
    if (block != 64 && block != 128 && block != 256 && block != 512 && block != 1024) return PF_ERANGE;
    // aggregation width: 0, or a power of two from block to 8 x block (the
    // vertices of one work item), at most 8192
    if (agg_width != 0 && (agg_width < block || agg_width > 8 * block || (agg_width & (agg_width - 1))))
        return PF_ERANGE;
    for (uint32_t v = 0; v < nviews; ++v) {
        const pf_status s = check_view(views[v]);
        if (s != PF_OK) return s;
        for (uint32_t u = 0; u < v; ++u)  // every view owns its tables
            if (views[u].cur.cell == views[v].cur.cell || views[u].cur.cell == views[v].prev.cell ||
                views[u].prev.cell == views[v].cur.cell)
                return PF_EINVAL;
    }
    uint64_t n[PF_MAX_VIEWS];
    uint32_t lg[PF_MAX_VIEWS];
    for (uint32_t v = 0; v < nviews; ++v) {
        n[v] = views[v].n;
        lg[v] = views[v].cur.log2_slots;
    }
    if (workspace_bytes < pfk::views_workspace_bytes(n, lg, nviews)) return PF_EINVAL;
    return launched(pfk::launch_views(views, nviews, block, agg_width, grid_per_cu, workspace, workspace_bytes,
                                      (hipStream_t)stream));
}

pf_status pf_microbench(int kind, void *buf, uint64_t bytes, uint32_t grain, uint32_t accesses_per_thread,
                        uint64_t seed, uint32_t *sink, void *stream) {
    if (kind < PF_MB_COPY || kind > PF_MB_CAS) return PF_ERANGE;
    if (!buf || !sink || (reinterpret_cast<uintptr_t>(buf) % 256) || !aligned(sink)) return PF_EINVAL;
    if (kind == PF_MB_COPY) {
        if (bytes < 32 || bytes % 32) return PF_ERANGE;
    } else {
        if (grain != 16 && grain != 32 && grain != 64) return PF_ERANGE;
        if (kind == PF_MB_RMW && grain != 32) return PF_ERANGE;
        if (bytes < grain || bytes % grain) return PF_ERANGE;
        const uint64_t granules = bytes / grain;
        if (granules & (granules - 1)) return PF_ERANGE;
        if (accesses_per_thread == 0) return PF_ERANGE;
    }
    return launched(pfk::launch_microbench(kind, buf, bytes, grain, (uint64_t)accesses_per_thread * PF_MB_THREADS,
                                           seed, sink, (hipStream_t)stream));
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
