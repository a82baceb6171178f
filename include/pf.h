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
 *      average over two sets of averages, or integrates them weighted by
 *      sample counts (Section 3.4.1).
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
 *   - n may be 0 (nothing is launched).  n is at most PF_MAX_VERTICES
 *     (2^31); larger n fails with PF_EINVAL.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_MAX_VERTICES 2147483648ull /* 2^31: vertex indices and launch sizes stay in 32 bits */

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
 *                  (PF_SUMS_FIXED64); with PF_SUMS_FLOAT32 the low 4 bytes of
 *                  each word hold a binary32 sum instead, the high 4 are 0
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
 * pf_table_carve().  Its 2^log2_slots slots are records of PF_SLOT_BYTES
 * bytes, so that a lookup reads one cache line per slot: the cell at offset
 * 0, the key at offset 32, the temporal value at offset 48, 8 bytes of
 * padding.  cell, key and blend point at slot 0's fields and advance by
 * PF_SLOT_BYTES per slot (key == (char *)cell + 32, blend == (char *)cell +
 * 48 or NULL for a table without temporal values, whose records keep the
 * space). */
#define PF_SLOT_BYTES 64
typedef struct pf_table {
    pf_cell *cell;       /* cells (fingerprint, count, fixed-point sums), stride PF_SLOT_BYTES */
    uint64_t *key;       /* full key of each occupied slot, written by the slot's claimer; stride PF_SLOT_BYTES */
    float *blend;        /* 4 floats per slot: temporal value rgb + count; stride PF_SLOT_BYTES; may be NULL */
    uint32_t *occ;       /* occupancy bitmap, 2^log2_slots / 32 words (bit s%32 of word s/32) */
    uint64_t *stats;     /* PF_STATS_LEN counters */
    uint32_t log2_slots; /* 4 .. 30 */
    uint32_t max_probe;  /* 1 .. 2^log2_slots: slots examined before PF_V_OVERFLOW */
    int32_t frac_bits;   /* 8 .. 40: fixed-point fraction bits of the sums */
    uint32_t sum_format; /* PF_SUMS_FIXED64 (set by pf_table_carve) or PF_SUMS_FLOAT32 */
} pf_table;

/* Sum formats.  PF_SUMS_FIXED64: exact int64 fixed-point sums; every
 * insertion order gives the same bits.  PF_SUMS_FLOAT32: the paper's own
 * accumulation (Section 3.3.1: one floating-point atomic add per component
 * of each vertex), binary32 sums whose rounding depends on the order in
 * which atomics arrive; each sum of n non-negative contributions is within
 * (n-1) 2^-24 / (1 - (n-1) 2^-24) of the exact sum, relative.  Float tables
 * are accepted by pf_insert_accumulate, pf_query_average,
 * pf_temporal_update and pf_mlp_train_step (frac_bits is then unused), and
 * rejected with PF_EINVAL by pf_insert_accumulate_binned and
 * pf_filter_views. */
#define PF_SUMS_FIXED64 0u
#define PF_SUMS_FLOAT32 1u

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
 * bytes, plus the cells of the last frame, not to the table size), the
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
 * On a PF_SUMS_FLOAT32 table the contribution is added as it is, with one
 * binary32 atomic add per component (no RADRANGE; a sum may overflow to
 * infinity), and combined lanes add in LDS first, in binary32 as well.
 * agg_width: 0 or 1 = one set of atomics per vertex; k = 2, 4, ..., 256 =
 * the lanes of each group of k consecutive threads of a 256-thread
 * workgroup that reach the same slot combine their contributions in LDS
 * first (they meet through 2k buckets indexed by the slot's low bits; a
 * lane whose bucket another slot took goes directly).
 * slot_out (nullable): receives the slot of each vertex (0xffffffff if
 * flagged) so that pf_query_average can skip probing.
 * Several batches may be inserted before one lookup.
 * Errors: PF_EINVAL, PF_ERANGE (agg_width above 256 or not a power of two). */
pf_status pf_insert_accumulate(const pf_table *t, const uint64_t *key, const float *r, const float *g,
                               const float *b, uint8_t *vflags, uint32_t *slot_out, uint64_t n,
                               uint32_t agg_width, void *stream);

/* [host] Workspace bytes of pf_insert_accumulate_binned for n vertices and a
 * table of 2^log2_slots slots; 0 when log2_slots > 25 (use
 * pf_insert_accumulate then). */
size_t pf_insert_workspace_bytes(uint64_t n, uint32_t log2_slots);

/* The same accumulation as pf_insert_accumulate (identical table, flags and
 * slots up to the order-dependent placement of probe collisions), without
 * device atomics on the cell sums: vertices are binned by the slot they
 * claim (a counting sort over tile histograms) and each bin -- a contiguous
 * slot range -- is summed in LDS by one workgroup, which then adds count and
 * sums to its cells with plain loads and stores and sets their occupancy
 * bits.  Compare-and-swap remains only for claiming new cells.
 * slot_out is required.  workspace: pf_insert_workspace_bytes(n, log2_slots)
 * device bytes (caller-owned, no alignment needed).
 * Errors: PF_EINVAL (NULL, misaligned, workspace too small, a
 * PF_SUMS_FLOAT32 table), PF_ERANGE (log2_slots > 25). */
pf_status pf_insert_accumulate_binned(const pf_table *t, const uint64_t *key, const float *r, const float *g,
                                      const float *b, uint8_t *vflags, uint32_t *slot_out, uint64_t n,
                                      void *workspace, size_t workspace_bytes, void *stream);

/* Key construction and the binned insert in one pass: the same keys, flags,
 * slots and table as pf_build_keys(px.., kp, t->log2_slots, key, NULL,
 * NULL, vflags) followed by pf_insert_accumulate_binned(t, key, r, g, b,
 * vflags, slot_out, ...), without the key and flag round trip through
 * memory between them.  key (nullable) receives the keys; vflags is
 * output only (0, PF_V_INVALID, PF_V_KEYRANGE, PF_V_RADRANGE or
 * PF_V_OVERFLOW per vertex); slot_out is required.  workspace as for
 * pf_insert_accumulate_binned.  Errors: those of the two calls. */
pf_status pf_build_keys_insert_binned(const pf_table *t, const float *px, const float *py, const float *pz,
                                      const float *nx, const float *ny, const float *nz, const uint8_t *valid,
                                      const pf_key_params *kp, const float *r, const float *g, const float *b,
                                      uint64_t n, uint64_t *key, uint8_t *vflags, uint32_t *slot_out,
                                      void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * keys, flags, slots and table as pf_build_keys_insert_binned, without a
 * workspace argument.  Its workspace is the library's own device array of
 * PF_NOALLOC_SCRATCH_BYTES, set up once per device at the first call on it
 * and held until the process ends; vertices go through it in consecutive
 * batches of at most PF_NOALLOC_BATCH (the insert accumulates, so the table
 * is the one a single call gives).  Never allocates or frees.  All calls on
 * one device share the array: calls that overlap in time on one device
 * (different streams, or host threads without ordering) race.
 * Errors: those of pf_build_keys_insert_binned except the workspace's;
 * PF_ERANGE (log2_slots > 25); PF_ELAUNCH (the array's address could not be
 * obtained, or a launch failed). */
#define PF_NOALLOC_SCRATCH_BYTES (80ull << 20)
#define PF_NOALLOC_BATCH (1u << 20)
pf_status pf_build_keys_insert_binned_noalloc(const pf_table *t, const float *px, const float *py, const float *pz,
                                              const float *nx, const float *ny, const float *nz, const uint8_t *valid,
                                              const pf_key_params *kp, const float *r, const float *g, const float *b,
                                              uint64_t n, uint64_t *key, uint8_t *vflags, uint32_t *slot_out,
                                              void *stream);

/* pf_build_keys_insert_binned followed by the temporal pass of the frame
 * (Section 3.4.1) in the same launches: the workgroup that owns a bin
 * of slots, once it has added the bin's records to its cells, computes each
 * cell's average and blends it with the value of the same key in prev (NULL:
 * no previous frame, the temporal value is the average), storing the
 * temporal value as pf_temporal_update (max_samples == 0: moving average with
 * alpha_old, mode 0) or pf_temporal_integrate (max_samples > 0) would; the
 * temporal-hit statistic is counted the same way.  Only the cells this call
 * inserts into get a temporal value, so t must be empty (initialised or
 * cleared) before the call: the frame's vertices are one batch.  prev must
 * be another table with the same log2_slots and temporal values.  Errors:
 * those of pf_build_keys_insert_binned; PF_EINVAL (t or prev without
 * temporal values, prev == t); PF_ERANGE (log2_slots differ, alpha_old
 * outside [0, 1] with max_samples == 0, max_samples > PF_MAX_SAMPLES). */
pf_status pf_build_keys_insert_binned_temporal(const pf_table *t, const float *px, const float *py,
                                               const float *pz, const float *nx, const float *ny,
                                               const float *nz, const uint8_t *valid, const pf_key_params *kp,
                                               const float *r, const float *g, const float *b, uint64_t n,
                                               uint64_t *key, uint8_t *vflags, uint32_t *slot_out,
                                               void *workspace, size_t workspace_bytes, const pf_table *prev,
                                               float alpha_old, uint32_t max_samples, void *stream);

/* ------------------------------------------------------------------ query */
/* Lookup (Sections 3.2, 3.3.1): for each vertex with vflags == 0, finds its
 * cell (from slot[i] when slot is non-NULL, else by probing with key[i]) and
 * writes avg_c = (float)((double)sum_c * 2^-frac_bits / (double)count)
 * (PF_SUMS_FLOAT32: sum_c / (float)count, one binary32 division), or
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

/* pf_query_average on t and pf_clear on another table `clear` in ONE launch:
 * a renderer alternating two tables across frames empties the table of the
 * frame before (read for the last time by the temporal pass) while it looks
 * up the current one, so the next frame's insert needs no clear of its own.
 * Results are those of the two calls.  `clear` must be another table whose
 * slots do not overlap t's, initialised and only modified through this
 * library; it is neither read nor written by the lookup.  Errors: those of
 * the two calls; PF_EINVAL also when clear is NULL or its slots overlap t's.
 * With n == 0 only the clear runs. */
pf_status pf_query_average_clear(const pf_table *t, const uint64_t *key, const uint32_t *slot,
                                 const float *r_in, const float *g_in, const float *b_in,
                                 const uint8_t *vflags, uint64_t n, int use_blend,
                                 float *r_out, float *g_out, float *b_out, uint32_t *count_out,
                                 const pf_table *clear, void *stream);

/* --------------------------------------------------------------- temporal */
/* Two sets of averages (Section 3.4.1).  For every occupied cell of `cur`
 * (found through its occupancy bitmap), computes c_new = sum / count as in
 * the lookup, searches its key in `prev` (fingerprint probe confirmed by the
 * stored 64-bit key) and stores into cur->blend the value c and a count N:
 *   mode 0 (moving average): c = alpha_old * c_old + (1 - alpha_old) * c_new
 *           (each product and the sum rounded to binary32; 1 - alpha_old
 *           rounded once), N = this frame's count;
 *   mode 1 (temporal integration): as pf_temporal_integrate with
 *           max_samples = PF_MAX_SAMPLES;
 * and c = c_new when the key is absent or prev is NULL.  Cells of prev that
 * do not occur in cur are dropped (prev holds the previous frame only).
 * The lookup with use_blend returns c and N as the vertex's count.
 * cur and prev must have the same log2_slots and both carry temporal values (blend not NULL).
 * Errors: PF_EINVAL (blend NULL), PF_ERANGE (alpha_old outside [0, 1]
 * in mode 0, unknown mode, differing sizes). */
pf_status pf_temporal_update(const pf_table *cur, const pf_table *prev, float alpha_old, int mode,
                             void *stream);
/* mode | PF_TEMPORAL_ACROSS_LEVELS: changes of resolution across frames
 * (Section 3.4.2).  A cell whose key is absent from prev takes, in this
 * order, its parent's value (the cell one level coarser that contains it:
 * level + 1, cell coordinates floor-divided by 2) with an eighth of the
 * parent's count as N_old (mode 1 skips a parent with fewer than 8), or its
 * children's (level - 1, coordinates 2x~ + 0 or 1 per axis) count-weighted
 * mean, (float)(sum_j N_j c_j / sum_j N_j) accumulated in double over
 * j = dx + 2 dy + 4 dz, with the sum of their counts as N_old; then the same
 * blend.  The temporal-hit statistic still counts exact keys only. */
#define PF_TEMPORAL_ACROSS_LEVELS 16

/* Temporal integration (Section 3.4.1): weighting the previous value by
 * alpha = N_old / (N_old + N_new), where N_old is its stored count and N_new
 * the cell's count in this frame, makes c the pooled mean of the samples of
 * both; the stored count is min(N_old + N_new, max_samples), so that once
 * the threshold is reached the history keeps a fixed weight (the paper's
 * heuristic of accumulating up to a number of samples).  Arithmetic:
 * alpha = N_old / (N_old + N_new) as one binary32 division of exact
 * integers, then c = alpha * c_old + (1 - alpha) * c_new as in mode 0.
 * Absent keys (or prev NULL): c = c_new, N = min(N_new, max_samples).
 * max_samples in [1, PF_MAX_SAMPLES].  Errors as pf_temporal_update. */
#define PF_MAX_SAMPLES 16777216u /* 2^24: counts stay exact in binary32 */
pf_status pf_temporal_integrate(const pf_table *cur, const pf_table *prev, uint32_t max_samples, void *stream);


/* ----------------------------------------------------------------- history */
/* Voxel values kept beyond the previous frame, with eviction by priority
 * (Section 3.4.3).  Direct-mapped: the voxel with key K lives only in slot
 * fmix64(K) mod 2^log2_slots (MurmurHash3's finaliser of the whole key).  A
 * slot holds a word, the key, the value (c: rgb, and N as the fourth float)
 * and the frame it was last written.  word = priority << 56 | (SplitMix64(K)
 * mod 2^56), priority = (min(age, 15) << 4) | (15 - min(floor(log2 N), 15)),
 * age = frames since written: of a slot's resident and the voxels of a
 * frame mapped to it, the smallest word stays (recent voxels first, then
 * those with more samples), so collisions and eviction are decided by one
 * atomic minimum and do not depend on the order of arrival.  An empty slot
 * has word = all ones.  Memory is bounded by 2^log2_slots slots of 32 bytes;
 * a voxel not written for more than max_age frames is dropped. */
typedef struct pf_history_slot {
    uint64_t word;  /* priority << 56 | key hash; all ones = empty */
    uint64_t key;
    float value[4]; /* rgb, N */
} pf_history_slot;  /* 32 bytes: one lookup reads one record */

typedef struct pf_history {
    pf_history_slot *slot; /* [2^log2_slots] */
    uint32_t *stamp;       /* [2^log2_slots] frame last written */
    uint32_t log2_slots;   /* 4 .. 30 */
    uint32_t max_age;      /* frames */
} pf_history;

/* [host] bytes of an arena for one history (256-byte aligned arrays). */
size_t pf_history_bytes(uint32_t log2_slots);
/* [host] points h's arrays into `arena`.  Errors: PF_EINVAL (NULL),
 * PF_ERANGE (log2_slots). */
pf_status pf_history_carve(void *arena, uint32_t log2_slots, uint32_t max_age, pf_history *h);
/* Empties every slot.  Errors: PF_EINVAL (NULL or misaligned arrays). */
pf_status pf_history_init(const pf_history *h, void *stream);

/* Temporal pass against the history instead of the previous frame's table,
 * for frame number `frame` (increasing by one per call; stamps are frame
 * numbers).  For every occupied cell of cur: c_new = sum / count as the
 * lookup computes it; if h's slot of its key holds that key, the blend of
 * pf_temporal_update (mode 0, alpha_old) or pf_temporal_integrate (mode 1,
 * max_samples) with the history's (c, N) as c_old and N_old, else c_new;
 * stored in cur->blend with its count as there.  Then h is aged to `frame`
 * (voxels whose age exceeds max_age are dropped, the others get the word of
 * their age), and the cells of cur compete for their slots with age 0 and
 * their stored count: the winner of a slot writes key, value (cur->blend)
 * and stamp.  The table's temporal-hit statistic counts the cells found.
 * Errors: PF_EINVAL (blend NULL, NULL history), PF_ERANGE (alpha_old,
 * mode, max_samples as in pf_temporal_update / pf_temporal_integrate). */
pf_status pf_temporal_history(const pf_table *cur, const pf_history *h, float alpha_old, int mode,
                              uint32_t max_samples, uint32_t frame, void *stream);

/* ------------------------------------------------- low-density fallbacks */
/* Section 3.3's fallbacks for voxels with a low number of vertices.  For
 * every occupied cell of t whose count in this frame is below `below`,
 * replaces the rgb of its temporal value (t->blend, written for every
 * occupied cell by pf_temporal_update / pf_temporal_integrate, which must
 * run first; with prev = NULL it holds the plain averages) by the pooled
 * average of a set of cells around it:
 *   PF_LD_NEIGHBOURS (0), neighbourhood search (Section 3.3.1): the cells
 *     of the 3 x 3 x 3 block of voxels at the same level and normal class
 *     whose quantised coordinates differ from its own by at most one per
 *     axis (itself included; coordinates outside the key range skipped);
 *   PF_LD_NORMALS (1), similar normals (Section 3.2.2, linear probing with
 *     the normal in the fingerprint only): the cells at the same position
 *     and level found along its probe run, from its home slot to the first
 *     empty slot (at most max_probe slots), whose normal class vector (-1,
 *     0, +1 per axis) has a positive dot product with its own.
 * Pooled value: (float)((double)S * 2^-frac_bits / (double)N) with S and N
 * the integer sums and counts of the set (S wraps modulo 2^64, which no
 * input within PF_V_RADRANGE reaches).  The stored count (blend's fourth
 * float) is kept, so the lookup still reports the cell's own count.
 * below <= 1 changes nothing.  Fixed-point tables only.
 * Errors: PF_EINVAL (blend NULL, binary32 sums), PF_ERANGE (mode). */
#define PF_LD_NEIGHBOURS 0
#define PF_LD_NORMALS 1
pf_status pf_low_density_fallback(const pf_table *t, uint32_t below, int mode, void *stream);

/* ---------------------------------------------- multi-level accumulation */
/* Section 3.3.2: accumulating at more than one resolution at a time.
 * pf_coarsen_keys writes, for every vertex, the key of the voxel `levels`
 * levels coarser that encloses its own: level field l' + levels, each cell
 * coordinate floor-divided by 2^levels, the same normal class.  This equals
 * Algorithm 1's quantisation floor(x' / (s * 2^(l' + levels))) of the same
 * jittered position (IEEE quotients by powers of two scale exactly).
 * vflags_out: the vertex's flag, except that PF_V_OVERFLOW (its key is
 * valid) becomes 0, and PF_V_KEYRANGE when l' + levels > 15; key_out is 0
 * for flagged vertices.  The coarse keys are then inserted into a second
 * table (pf_insert_accumulate[_binned]) and optionally blended across
 * frames (pf_temporal_update) like the vertex's own.  levels in [1, 31].
 * Errors: PF_EINVAL (NULL or misaligned arrays, n > PF_MAX_VERTICES),
 * PF_ERANGE (levels). */
pf_status pf_coarsen_keys(const uint64_t *key, const uint8_t *vflags, uint64_t n, uint32_t levels,
                          uint64_t *key_out, uint8_t *vflags_out, void *stream);

/* The lookup of multi-level accumulation: as pf_query_average through
 * `slot` in `fine`, except that a vertex whose cell's count (the count the
 * lookup returns: blend's count with use_blend, else the cell's) is below
 * `below` takes the value and count of its coarse cell (slot_coarse in
 * `coarse`) when that vertex was placed there (vflags_coarse == 0 and a
 * valid slot).  Flagged vertices (vflags != 0) write their own contribution
 * and count 0.  r_out.. may alias r_in..; count_out is nullable.
 * Errors: PF_EINVAL (NULL or misaligned arrays, NULL blend with use_blend). */
pf_status pf_query_multilevel(const pf_table *fine, const pf_table *coarse, const uint32_t *slot,
                              const uint32_t *slot_coarse, const float *r_in, const float *g_in,
                              const float *b_in, const uint8_t *vflags, const uint8_t *vflags_coarse,
                              uint64_t n, uint32_t below, int use_blend, float *r_out, float *g_out,
                              float *b_out, uint32_t *count_out, void *stream);

/* ----------------------------------------------------------- pixel resolve */
/* Section 3: after filtering, each selected vertex's value (r, g, b: the
 * lookup's output) is multiplied by its throughput (tr, tg, tb: the
 * attenuation from the camera along its path up to the vertex) and
 * accumulated in its pixel.  Vertices are bounce-major: vertex k of pixel p
 * is at k * pixels + p, k < verts_per_path.  Per pixel and channel, in
 * binary32 with each product and sum rounded, k = 0, 1, ...:
 * acc = acc + t * c over the vertices with valid != 0 (valid NULL: all);
 * t = 1 when tr, tg, tb are NULL (all three or none).  accumulate != 0
 * starts from the pixel's current value, else from 0.
 * Errors: PF_EINVAL (NULL or misaligned arrays, pixels * verts_per_path >
 * PF_MAX_VERTICES, throughput arrays partly NULL). */
pf_status pf_resolve_pixels(const float *r, const float *g, const float *b, const float *tr, const float *tg,
                            const float *tb, const uint8_t *valid, uint64_t pixels, uint32_t verts_per_path,
                            int accumulate, float *pr, float *pg, float *pb, void *stream);

/* ------------------------------------------------------- learned fallback */
/* A small BF16 network that predicts the contribution of vertices whose
 * cell holds few samples, trained online on the averages of well-populated
 * cells.  It is not part of the paper; it stands where Section 3.3 puts its
 * fallbacks for voxels with a low number of vertices.
 *
 * Network: x [80] -> 64 (ReLU) -> 64 (ReLU) -> 3, i.e.
 *   z1 = W1 x + b1, a1 = relu(z1), z2 = W2 a1 + b2, a2 = relu(z2),
 *   y = W3 a2 + b3.
 * Parameters, FP32, packed in this order (PF_MLP_NPARAM floats):
 *   W1 [64][80], b1 [64], W2 [64][64], b2 [64], W3 [16][64], b3 [16];
 *   rows 3..15 of W3 and entries 3..15 of b3 are padding and must be 0.
 * Features of a vertex with key k (cell index x~, level l'), position x,
 * normal n and camera p_cam:
 *   p_c = (x~_c + 1/2) * 2^(l' - 10)   (the cell centre in units of s, exact)
 *   x[6j + c] = sin(pi 2^j p_c), x[6j + 3 + c] = cos(pi 2^j p_c), j = 0..11
 *   x[72 + c] = n_c, x[75 + c] = (x - p_cam)_c / |x - p_cam|, x[78..79] = 0
 * evaluated in FP64 and rounded FP64 -> FP32 -> BF16 (nearest even), with
 * zero results taken as +0.
 * Arithmetic: BF16 operands (features, a BF16 copy of the weights, a1, a2 and
 * the back-propagated gradients gy, gz2, gz1) on MFMA with FP32
 * accumulation; biases, loss and gradient sums in FP32.  Loss: mean over the
 * batch and the 3 channels of (y - target)^2.  Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8) on the FP32 weights. */
#define PF_MLP_IN 80
#define PF_MLP_HIDDEN 64
#define PF_MLP_NPARAM 10384
#define PF_MLP_BLOCK_SAMPLES 64   /* training batch granularity */

typedef struct pf_mlp {
    float *w;            /* [PF_MLP_NPARAM] FP32 weights (caller fills before pf_mlp_init) */
    uint16_t *wb;        /* [PF_MLP_NPARAM] BF16 copy used by the products (16-byte aligned) */
    float *m;            /* [PF_MLP_NPARAM] Adam first moment */
    float *v;            /* [PF_MLP_NPARAM] Adam second moment */
    float *partial;      /* [max_batch / 64][PF_MLP_NPARAM + 1] per-workgroup gradient and loss sums */
    float *loss;         /* [1] mean loss of the last training step */
    uint32_t max_batch;  /* multiple of 64 */
    uint32_t reserved;
} pf_mlp;

/* Per-view geometry the features are computed from (device pointers, n
 * vertices each; cam by value). */
typedef struct pf_geometry {
    const uint64_t *key;
    const float *px, *py, *pz;
    const float *nx, *ny, *nz;
    float cam[3];
    float reserved;
} pf_geometry;

/* [host] Arena bytes for a network trained with batches up to max_batch. */
size_t pf_mlp_bytes(uint32_t max_batch);

/* [host] Carves *m out of `arena` (pf_mlp_bytes(max_batch) bytes).
 * Errors: PF_EINVAL (NULL), PF_ERANGE (max_batch 0, not a multiple of 64,
 * or above 2^20). */
pf_status pf_mlp_carve(void *arena, uint32_t max_batch, pf_mlp *m);

/* Zeroes the Adam moments and the loss and rounds the FP32 weights (already
 * written to m->w by the caller) into the BF16 copy. */
pf_status pf_mlp_init(const pf_mlp *m, void *stream);

/* [host] Workspace bytes of pf_mlp_select for n vertices. */
size_t pf_mlp_select_workspace_bytes(uint64_t n);

/* Lists, in ascending vertex order, the vertices with vflags == 0 whose
 * cell count (from pf_query_average's count_out) is >= train_from
 * (train_idx) and those whose count is < sparse_below (sparse_idx); writes
 * the two list lengths to counts[0] and counts[1] (device).  Lists hold up to
 * n entries each.  Workspace: pf_mlp_select_workspace_bytes(n) device bytes.
 * Errors: PF_EINVAL (NULL, misaligned, n too large). */
pf_status pf_mlp_select(const uint8_t *vflags, const uint32_t *count, uint64_t n, uint32_t sparse_below,
                        uint32_t train_from, uint32_t *train_idx, uint32_t *sparse_idx, uint32_t *counts,
                        void *workspace, void *stream);

/* One training step on `batch` samples (a multiple of 64, <= max_batch).
 * Sample j is vertex train_idx[(u * counts[0]) >> 32] with u the first
 * output of PCG32 seeded with (seed, j); its target is the plain average
 * (sum / count, as in the lookup) of its cell in table t at slot[vertex]
 * (pf_insert_accumulate's slot_out).  Computes the loss gradient in fixed
 * order (deterministic), then one Adam step with bias corrections for step
 * number `step` (>= 1) and learning rate lr, and refreshes the BF16 copy.
 * A step with counts[0] == 0 changes nothing.
 * Errors: PF_EINVAL (NULL), PF_ERANGE (batch, step, lr). */
pf_status pf_mlp_train_step(const pf_mlp *m, const pf_table *t, const pf_geometry *g, const uint32_t *slot,
                            const uint32_t *train_idx, const uint32_t *counts, uint32_t batch, uint64_t seed,
                            uint32_t step, float lr, void *stream);

/* The network's input features (BF16 bit patterns, [n][PF_MLP_IN]) of the
 * n vertices listed in idx, as the training and inference kernels compute
 * them.  For inspection and tests.
 * Errors: PF_EINVAL (NULL, misaligned), PF_ERANGE (n * PF_MLP_IN >= 2^32). */
pf_status pf_mlp_features(const pf_geometry *g, const uint32_t *idx, uint64_t n, uint16_t *out, void *stream);

/* Inference for the counts[1] vertices listed in sparse_idx (n_max bounds
 * the list): y = network(features); when all three outputs are finite the
 * vertex's r, g, b become max(0, y_c), otherwise they are left unchanged.
 * Errors: PF_EINVAL (NULL, misaligned), PF_ERANGE (n_max too large). */
pf_status pf_mlp_infer(const pf_mlp *m, const pf_geometry *g, const uint32_t *sparse_idx, const uint32_t *counts,
                       uint64_t n_max, float *r, float *gch, float *b, void *stream);


/* ----------------------------------------------------------- many views */
/* One view of a batched launch: its vertex streams (SoA, n each), its
 * outputs, its key parameters and its tables.  Tables of all views may be
 * carved from one arena. */
typedef struct pf_view {
    const float *px, *py, *pz, *nx, *ny, *nz;
    const uint8_t *valid;     /* nullable */
    const float *r, *g, *b;   /* contributions */
    uint64_t *key;            /* [n] out, nullable (8 bytes a vertex that only callers reading the keys need) */
    uint8_t *vflags;          /* [n] out */
    uint32_t *slot;           /* [n] out: cell of each vertex, 0xffffffff if unfiltered */
    float *r_out, *g_out, *b_out;  /* [n] out; must not alias r, g, b */
    uint32_t *count_out;      /* [n] out, nullable */
    pf_table cur;             /* cleared, then filled by this launch */
    pf_table prev;            /* previous frame (read, then emptied); prev.cell == NULL: none */
    pf_key_params kp;
    uint32_t n;               /* vertices (at most PF_MAX_VERTICES) */
    float alpha_old;          /* moving-average weight of the previous value */
    int32_t temporal;         /* 1: lookup returns the moving average (cur needs temporal values: blend not NULL) */
    uint32_t reserved;
} pf_view;

#define PF_MAX_VIEWS 64

/* [host] Device workspace bytes of pf_filter_views for nviews views of n[v]
 * vertices and tables of 2^log2_slots[v] slots (host arrays), enough for
 * every workgroup size: barrier counters, the device copy of the
 * descriptors, and per view the records of its insert (32 bytes, about two
 * per vertex) with their bucket counts.  0 for bad arguments. */
size_t pf_views_workspace_bytes(const uint64_t *n, const uint32_t *log2_slots, uint32_t nviews);

/* [host] Device workspace bytes of pf_filter_views_concurrent: the binned
 * insert's workspace of every view (pf_insert_workspace_bytes), each
 * 256-byte aligned.  0 for bad arguments. */
size_t pf_views_concurrent_workspace_bytes(const uint64_t *n, const uint32_t *log2_slots, uint32_t nviews);

/* The frame of pf_filter_views (same descriptors, the same results bit for
 * bit) with each view through the single-view calls: pf_clear(cur), then
 * pf_build_keys_insert_binned_temporal with prev (NULL when prev.cell is
 * NULL) and alpha_old, or pf_build_keys_insert_binned when temporal is 0,
 * then pf_query_average_clear emptying prev, or pf_query_average when there
 * is no prev.  The views go to the library's streams of the current device
 * (created at the first call, default priority), which wait on an event
 * recorded on `stream`; the largest views first, each to the stream with the
 * fewest vertices so far, so that small views run beside large ones; then
 * `stream` waits on an event of every library stream.  Calls are serialised
 * on the host per device.  workspace: pf_views_concurrent_workspace_bytes
 * device bytes, 256-byte aligned.
 * Errors: those of pf_filter_views (not block, agg_width, grid_per_cu). */
pf_status pf_filter_views_concurrent(const pf_view *views, uint32_t nviews, uint32_t nstreams, void *workspace,
                                     size_t workspace_bytes, void *stream);

/* Filters nviews views in ONE persistent launch (a cooperative grid of
 * resident workgroups of `block` threads), in four phases separated by
 * grid-wide barriers, the work items of all views spread over all
 * workgroups:
 *   clear      every view's `cur` and its bucket counts;
 *   insert     keys of every vertex (as pf_build_keys) and its cell
 *              (Sections 3.2, 3.3.1): agg_width 0 claims the cell and adds
 *              count and sums with one set of device atomics per vertex;
 *              otherwise each workgroup merges windows of agg_width
 *              consecutive vertices by key in an LDS table of
 *              min(agg_width, 4 x block, 1536) entries (a vertex that finds
 *              no room goes alone), and each group claims its cell once and
 *              writes one record {slot, count, sums} into the bucket of its
 *              bin of min(2 x block, 2048) slots (a full bucket adds the
 *              group with device atomics instead);
 *   reduce     per bin, the records summed and added to the cells by one
 *              workgroup, then, when temporal is set, the temporal values of
 *              the bin's cells (as pf_temporal_update, mode 0, Section 3.4.1);
 *   lookup     every vertex (as pf_query_average with the slots), and,
 *              in the same phase, `prev` emptied (as pf_clear): the temporal
 *              blend has read it for the last time, so that a caller who
 *              alternates two tables finds the next frame's `cur` empty and
 *              the next launch's clear costs nothing.
 * Results equal those of the single-view calls (integer sums).
 * views: [host] array of nviews descriptors, validated on the host and
 * copied into the workspace before the call returns.  block in
 * {64, 128, 256, 512, 1024}; agg_width 0 or a power of two from block to
 * 8 x block; grid_per_cu: workgroups per compute unit (0 = as many as fit).
 * workspace: pf_views_workspace_bytes(n, log2_slots, nviews) device bytes
 * (workspace_bytes gives its size), 256-byte aligned; its first uint32 is a
 * status word, non-zero if a barrier wait ever exceeded its bound (every
 * workgroup then stops; with a cooperative launch all workgroups are
 * resident, so it stays 0); the next words hold the grid size and, after a
 * timed-out wait, the arrivals that were seen; words 4..13 hold five 64-bit
 * wall-clock readings of workgroup 0 (start, end of clear, of insert, of
 * reduce, of its own lookup), in ticks of pf_wall_clock_hz().
 * Errors: PF_EINVAL (NULL, misaligned, inconsistent descriptor, a
 * PF_SUMS_FLOAT32 table, workspace too small), PF_ERANGE (nviews 0 or above
 * PF_MAX_VIEWS, block, agg_width, parameters), PF_ELAUNCH. */
pf_status pf_filter_views(const pf_view *views, uint32_t nviews, uint32_t block, uint32_t agg_width,
                          uint32_t grid_per_cu, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------ diagnostics */
/* ------------------------------------------------------------ diagnostics */
/* Memory-system probe giving the filter's rooflines measured denominators
 * (not a step of the method).  PF_MB_COPY copies the first half of buf to
 * the second.  The other kinds make accesses_per_thread * PF_MB_THREADS
 * accesses, each to a granule of `grain` bytes chosen at random (fmix64 of
 * seed and the access number) among the bytes / grain granules of buf:
 *   PF_MB_GATHER   reads the granule
 *   PF_MB_SCATTER  writes the granule
 *   PF_MB_RMW      adds to a 32-byte cell's count and three sums with the
 *                  insert's device atomics (u32 + 3 x u64; grain 32)
 *   PF_MB_CAS      compares-and-swaps the granule's first word
 * buf (256-byte aligned) is overwritten; bytes / grain must be a power of
 * two (PF_MB_COPY: bytes a multiple of 32).  sink: one device uint32 that
 * keeps the reads alive (practically never written).
 * Errors: PF_EINVAL (NULL, misaligned), PF_ERANGE (kind, grain, bytes,
 * accesses_per_thread 0). */
#define PF_MB_COPY 0
#define PF_MB_GATHER 1
#define PF_MB_SCATTER 2
#define PF_MB_RMW 3
#define PF_MB_CAS 4
#define PF_MB_THREADS 2097152u
pf_status pf_microbench(int kind, void *buf, uint64_t bytes, uint32_t grain, uint32_t accesses_per_thread,
                        uint64_t seed, uint32_t *sink, void *stream);

/* Derives USED, DISP and HIST from the table (occupancy bitmap and keys),
 * copies the PF_STATS_LEN counters to host memory and waits for the copy.
 * The only call that blocks the host. */
pf_status pf_read_stats(const pf_table *t, uint64_t *host_out, void *stream);

/* [host] Frequency of the current device's wall clock (the stamps of
 * pf_filter_views), in Hz; 0 if it cannot be queried. */
uint64_t pf_wall_clock_hz(void);

/* Library version string [host]. */
const char *pf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
