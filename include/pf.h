/*
 * pf.h -- C ABI of the MI355X (gfx950) hot path of hashed path space
 * filtering (Binder, Fricke, Keller, "Massively Parallel Path Space
 * Filtering").
 *
 * For every path vertex the library
 *   1. derives a level of detail from the distance to the camera,
 *   2. jitters the position in the tangent plane and quantises position,
 *      level and normal class into a 64-bit key with a 32-bit fingerprint
 *      (Algorithm 1, Sections 3.1.2-3.1.4 and 3.2.1),
 *   3. inserts the key into an open-addressing hash table with linear probing
 *      while accumulating the vertex's contribution and a counter
 *      (Section 3.2; the voxel average of Eq. (8) with w = 1),
 *   4. looks up its cell and replaces its contribution by the cell average,
 *      sum divided by counter (Sections 3.2 and 3.3.1),
 *   5. blends cell averages across frames with an exponential moving
 *      average over two sets of averages (Section 3.4.1).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless marked [host].  The library never
 *     allocates, frees or synchronises, except pf_read_stats (which waits for
 *     its own copy).  The caller owns all memory.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and runs asynchronously.  Calls that touch the same table must be
 *     ordered on one stream; calls on different tables are independent.
 *   - Argument checks run on the host before anything is enqueued and return
 *     a negative status; nothing is launched then.  Per-vertex conditions
 *     never fail a call: they are reported in the per-vertex flags.
 *   - Vertex arrays are structure-of-arrays, n elements each, naturally
 *     aligned (4 bytes for float/uint32, 8 for uint64).
 *   - n may be 0 (nothing is launched).  n must be below 2^32.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef int pf_status;
#define PF_OK 0
#define PF_EINVAL (-1)   /* NULL or misaligned pointer, n too large */
#define PF_ERANGE (-2)   /* a parameter outside its documented range */
#define PF_ELAUNCH (-3)  /* the HIP runtime rejected a launch or copy */

/* ----------------------------------------------------------- vertex flags */
/* One byte per vertex.  A vertex with any flag set is "unfiltered": the
 * lookup returns its own contribution and a count of 0 (the fallback the
 * paper prescribes when linear probing exceeds its step limit). */
#define PF_V_INVALID 1u   /* valid[i] == 0, or a non-finite position, normal or contribution */
#define PF_V_KEYRANGE 2u  /* some |x~_c| >= 2^16: the key cannot hold the cell index */
#define PF_V_OVERFLOW 4u  /* no matching or free slot within max_probe steps */
#define PF_V_RADRANGE 8u  /* some |contribution * 2^frac_bits| >= 2^62 */

/* ------------------------------------------------------------------ table */
/* Slot layout (one cell per slot, 32 bytes, 32-byte aligned):
 *   uint32 fp      fingerprint of the key stored here, 0 = empty (the
 *                  sentinel of Section 3.2.1)
 *   uint32 count   vertices accumulated in this cell
 *   int64  sum[3]  contributions in fixed point, sum of rint(c * 2^frac_bits)
 * The fingerprint sits in the cell so that probing and accumulating touch
 * one memory line. */
typedef struct pf_cell {
    uint32_t fp;
    uint32_t count;
    int64_t sum[3];
} pf_cell;

/* Statistics block: PF_STATS_LEN uint64 counters.  The kernels never update
 * one shared counter per cell or per vertex (device atomics on one address
 * serialise): USED, DISP and HIST are derived from the table by
 * pf_read_stats, and OVERFLOW and TEMPORAL_HIT are gathered in spread partial
 * counters that pf_read_stats folds in.  Read them only through
 * pf_read_stats. */
#define PF_STAT_USED 0        /* occupied slots (= distinct cells inserted) */
#define PF_STAT_DISP 1        /* sum over occupied slots of (slot - home) mod 2^m */
#define PF_STAT_OVERFLOW 2    /* vertices flagged PF_V_OVERFLOW by insert */
#define PF_STAT_TEMPORAL_HIT 3 /* cells that found their key in the previous table */
#define PF_STAT_HIST 8        /* [65]: occupied slots by displacement, bin 64 = displacement >= 64 */
#define PF_STAT_PART_HIT 80   /* [32] internal partial counters */
#define PF_STAT_PART_OVF 112  /* [16] internal partial counters */
#define PF_STATS_LEN 128

/* A table is a set of views into one caller-owned arena, filled in by
 * pf_table_carve().  cell, key and blend have 2^log2_slots entries. */
typedef struct pf_table {
    pf_cell *cell;       /* cells (fingerprint, count, fixed-point sums) */
    uint64_t *key;       /* full key of each occupied slot, written by the slot's claimer */
    float *blend;        /* 4 floats per slot: temporal value rgb + count; may be NULL */
    uint32_t *occ;       /* occupancy bitmap, 2^log2_slots / 32 words (bit s%32 of word s/32) */
    uint64_t *stats;     /* PF_STATS_LEN counters */
    uint32_t log2_slots; /* 4 .. 30 */
    uint32_t max_probe;  /* 1 .. 2^log2_slots: slots examined before PF_V_OVERFLOW */
    int32_t frac_bits;   /* 8 .. 40: fixed-point fraction bits of the sums */
    uint32_t reserved;
} pf_table;

/* [host] Bytes of one table arena (including 256 bytes of alignment slack). */
size_t pf_table_bytes(uint32_t log2_slots, int with_blend);

/* [host] Fills *t with views into `arena` (device memory of at least
 * pf_table_bytes(log2_slots, with_blend) bytes).  Nothing is enqueued.
 * Errors: PF_EINVAL (NULL), PF_ERANGE (log2_slots, max_probe, frac_bits). */
pf_status pf_table_carve(void *arena, uint32_t log2_slots, int with_blend, uint32_t max_probe,
                         int32_t frac_bits, pf_table *t);

/* Zeroes every cell, the occupancy bitmap and the statistics of a freshly
 * carved table.  Must run once before the first pf_clear() or insert. */
pf_status pf_table_init(const pf_table *t, void *stream);

/* Empties a table for the next frame: zeroes the cells whose occupancy bit
 * is set (work proportional to the occupancy bitmap, 2^log2_slots / 8
 * bytes, plus the cells of the last frame, not to the cell array), the
 * bitmap and the statistics.  The table must have been initialised and only
 * modified through this library since. */
pf_status pf_clear(const pf_table *t, void *stream);

/* ------------------------------------------------------------------- keys */
/* Per-view key parameters (passed by host pointer). */
typedef struct pf_key_params {
    float cam[3];       /* camera position p_cam */
    float s;            /* scale: cell edge is s * 2^level (Algorithm 1), > 0 and finite */
    uint64_t seed;      /* jitter seed of this frame (PCG32 initial state) */
    uint64_t idx_base;  /* PCG32 stream of vertex i is idx_base + i */
} pf_key_params;

/* Key construction of Algorithm 1 for n vertices.
 *   l  = level_of_detail(|p_cam - x|) = floor(log2 d), with d^2 evaluated
 *        as (dx*dx + dy*dy) + dz*dz in binary32, clamped to [-16, 15]
 *        (-16 when d^2 is zero or subnormal);
 *   r  = three PCG32 (XSH-RR) outputs of stream idx_base + i seeded with
 *        `seed`, each mapped to (u >> 8) * 2^-24 - 1/2;
 *   x' = x + (r - (r.n) n) * (s * 2^l)           (jitter in the tangent plane)
 *   l' = level_of_detail(|p_cam - x'|)
 *   x~ = floor(x' / (s * 2^l'))                   (IEEE binary32 division)
 *   key = (x~_x + 2^16) | (x~_y + 2^16) << 17 | (x~_z + 2^16) << 34
 *         | (l' + 16) << 51 | class << 56, where class has 2 bits per axis:
 *         1 if n_c > 0, 2 if n_c < 0, 0 if n_c == 0.
 *   home = fmix64(key & (2^56 - 1)) mod 2^log2_slots (MurmurHash3's
 *          finaliser; the normal class is not part of the home index)
 *   fp   = high 32 bits of SplitMix64(key), 0 replaced by 1.
 * All float arithmetic is binary32, round to nearest, without contraction,
 * so results are bit-reproducible.
 * Inputs: px..nz positions and unit normals; valid (nullable: all valid).
 * Outputs: key[n]; fp[n] and home[n] (each nullable, for inspection);
 * vflags[n] set to 0, PF_V_INVALID or PF_V_KEYRANGE.  Flagged vertices get
 * key = fp = home = 0.
 * Errors: PF_EINVAL (NULL/misaligned), PF_ERANGE (log2_slots, s). */
pf_status pf_build_keys(const float *px, const float *py, const float *pz,
                        const float *nx, const float *ny, const float *nz,
                        const uint8_t *valid, uint64_t n, const pf_key_params *kp,
                        uint32_t log2_slots, uint64_t *key, uint32_t *fp, uint32_t *home,
                        uint8_t *vflags, void *stream);

/* ----------------------------------------------------------------- insert */
/* Accumulation (Section 3.2): every vertex with vflags == 0 converts its
 * contribution (r, g, b) to fixed point q_c = rint(c * 2^frac_bits), probes
 * from home(key) for a cell whose fingerprint equals fp(key) or claims the
 * first empty cell with a compare-and-swap (recording the key and setting
 * the slot's occupancy bit), and adds 1 to the counter and q to the sums with
 * device-scope integer atomics.  Integer sums make the result independent of
 * the order in which vertices arrive.
 * Vertices with non-finite contributions get PF_V_INVALID, with out-of-range
 * ones PF_V_RADRANGE, those finding neither within max_probe slots
 * PF_V_OVERFLOW; vertices already flagged are skipped.
 * agg_width: 0 = one set of atomics per vertex; k > 0 = lanes of a wavefront
 * that reach the same slot combine their contributions first (at most k
 * distinct slots per wavefront are combined, the rest go directly).
 * slot_out (nullable): receives the slot of each vertex (0xffffffff if
 * flagged) so that pf_query_average can skip probing.
 * Several batches may be inserted before one lookup.
 * Errors: PF_EINVAL, PF_ERANGE (agg_width > 64). */
pf_status pf_insert_accumulate(const pf_table *t, const uint64_t *key, const float *r, const float *g,
                               const float *b, uint8_t *vflags, uint32_t *slot_out, uint64_t n,
                               uint32_t agg_width, void *stream);

/* ------------------------------------------------------------------ query */
/* Lookup (Sections 3.2, 3.3.1): for each vertex with vflags == 0, finds its
 * cell (from slot[i] when slot is non-NULL, else by probing with key[i]) and
 * writes avg_c = (float)((double)sum_c * 2^-frac_bits / (double)count), or
 * the cell's temporal value when use_blend != 0 (after pf_temporal_update).
 * Flagged vertices, and vertices whose key is not found, write their own
 * contribution and count 0.  r_out.. may alias r_in.. (in-place update);
 * then flagged vertices are not written at all.  count_out is nullable.
 * Errors: PF_EINVAL (NULL key and slot; NULL blend with use_blend). */
pf_status pf_query_average(const pf_table *t, const uint64_t *key, const uint32_t *slot,
                           const float *r_in, const float *g_in, const float *b_in,
                           const uint8_t *vflags, uint64_t n, int use_blend,
                           float *r_out, float *g_out, float *b_out, uint32_t *count_out,
                           void *stream);

/* --------------------------------------------------------------- temporal */
/* Two sets of averages (Section 3.4.1).  For every occupied cell of `cur`
 * (found through its occupancy bitmap),
 * computes c_new = sum / count as in the lookup, searches its key in `prev`
 * (fingerprint probe confirmed by the stored 64-bit key) and stores
 *   mode 0: c = alpha_old * c_old + (1 - alpha_old) * c_new  (each product
 *           and the sum rounded to binary32; 1 - alpha_old rounded once),
 *           or c = c_new when the key is absent or prev is NULL,
 * into cur->blend together with the count.  Cells of prev that do not
 * occur in cur are dropped (prev holds the previous frame only).
 * cur and prev must have the same log2_slots and both carry blend arrays.
 * Errors: PF_EINVAL (no blend array), PF_ERANGE (alpha_old outside [0, 1],
 * unknown mode, differing sizes). */
pf_status pf_temporal_update(const pf_table *cur, const pf_table *prev, float alpha_old, int mode,
                             void *stream);

/* ------------------------------------------------------------ diagnostics */
/* Derives USED, DISP and HIST from the table (occupancy bitmap and keys),
 * copies the PF_STATS_LEN counters to host memory and waits for the copy.
 * The only call that blocks the host. */
pf_status pf_read_stats(const pf_table *t, uint64_t *host_out, void *stream);

/* Library version string [host]. */
const char *pf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
