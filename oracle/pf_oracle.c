/*
 * Plain CPU oracle of hashed path space filtering.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * statement of what the GPU path must compute.  It shares no code, header,
 * table or constant with the GPU library; only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load it.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared
 *        (x86-64 SSE arithmetic: every float operation is rounded to IEEE
 *        binary32 on its own; no fused multiply-add.)
 *
 * What it computes (per view and frame), following the paper:
 *   - key construction of Algorithm 1 (Section 3.2.1): level of detail at x,
 *     jitter in the tangent plane (Section 3.1.4) scaled by s * 2^l, level of
 *     detail again at the jittered x', quantisation floor(x' / (s * 2^l')),
 *     normal classes (Section 3.1.2), the home index from a first hash and a
 *     fingerprint from a second, different hash with 0 reserved as the empty
 *     sentinel (Section 3.2.1);
 *   - the voxel average of Eq. (8) with w = 1 as an exact group-by on the
 *     key (the "gather" formulation of Section 3.2), radiance summed in
 *     fixed point with 64-bit integers;
 *   - a sequential simulation of linear probing with a step limit (Section
 *     3.2) that yields the insertion-order-free facts of the table;
 *   - the lookup "sum divided by counter" (Sections 3.2 and 3.3.1) with the
 *     unfiltered contribution as fallback for vertices that could not be
 *     placed;
 *   - the exponential moving average of Section 3.4.1 over two sets of
 *     averages, and its temporal integration with a sample-count threshold;
 *   - the fallbacks of Section 3.3 for voxels with few vertices: the pooled
 *     average of the neighbouring voxels, or of the voxels with a similar
 *     normal in the same probe run; and the keys of coarser voxels for
 *     multi-level accumulation (Section 3.3.2).
 *
 * Readings of points the paper leaves open (each stated where it is used):
 *   level_of_detail(d) = floor(log2 d) computed as floor(floor(log2 d2)/2)
 *   from the binary32 value d2 = (dx*dx + dy*dy) + dz*dz, clamped to
 *   [-16, 15], and -16 for d2 == 0; jitter = r - (r.n) n with r uniform in
 *   [-1/2, 1/2)^3 from PCG32 (O'Neill 2014) seeded with (seed, idx_base+i);
 *   normal class per axis: 1 if n > 0, 2 if n < 0, 0 if n == 0;
 *   home = MurmurHash3 fmix64(position part of the key) mod 2^m;
 *   fingerprint = high 32 bits of the SplitMix64 output function of the key,
 *   0 mapped to 1; fixed point q = rint(r * 2^F), F = frac_bits;
 *   average = (float)((double)S * 2^-F / (double)count).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#if !defined(__FLT_EVAL_METHOD__) || __FLT_EVAL_METHOD__ != 0
#error "the oracle needs binary32 evaluation of float expressions (x86-64 SSE)"
#endif

/* per-vertex flags (values are part of the documented interface) */
enum { ORC_INVALID = 1, ORC_KEYRANGE = 2, ORC_OVERFLOW = 4, ORC_RADRANGE = 8 };

enum { ORC_LMIN = -16, ORC_LMAX = 15, ORC_QMAX = 65536 /* |x~| < 2^16 */ };

/* ---------------------------------------------------------------------- */
/* PCG32, "PCG: A Family of Simple Fast Space-Efficient Statistically Good
 * Algorithms for Random Number Generation", M. E. O'Neill, 2014:
 * 64-bit LCG state with multiplier 6364136223846793005 and an odd increment
 * selecting the stream, output permutation XSH-RR (xorshift high, random
 * rotation), and the standard seeding (state 0, step, add initstate, step). */
typedef struct { uint64_t state, inc; } orc_pcg32;

static uint32_t orc_pcg32_next(orc_pcg32 *g)
{
    uint64_t old = g->state;
    g->state = old * 6364136223846793005ULL + g->inc;
    uint32_t xorshifted = (uint32_t)(((old >> 18) ^ old) >> 27);
    uint32_t rot = (uint32_t)(old >> 59);
    return (xorshifted >> rot) | (xorshifted << ((32u - rot) & 31u));
}

static void orc_pcg32_seed(orc_pcg32 *g, uint64_t initstate, uint64_t initseq)
{
    g->state = 0;
    g->inc = (initseq << 1) | 1u;
    orc_pcg32_next(g);
    g->state += initstate;
    orc_pcg32_next(g);
}

/* exposed for the published-output test of the generator */
void orc_pcg32_outputs(uint64_t initstate, uint64_t initseq, uint32_t count, uint32_t *out)
{
    orc_pcg32 g;
    orc_pcg32_seed(&g, initstate, initseq);
    for (uint32_t i = 0; i < count; ++i) out[i] = orc_pcg32_next(&g);
}

/* first output of the generator seeded with (initstate, stream j), j = 0..n-1 */
void orc_pcg32_first(uint64_t initstate, uint64_t n, uint32_t *out)
{
    for (uint64_t j = 0; j < n; ++j) {
        orc_pcg32 g;
        orc_pcg32_seed(&g, initstate, j);
        out[j] = orc_pcg32_next(&g);
    }
}

/* MurmurHash3's 64-bit finaliser (Appleby, public domain). */
uint64_t orc_fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

/* SplitMix64 output for state x (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): add the golden gamma, then
 * the variant-13 mix. */
uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* ---------------------------------------------------------------------- */
/* Key construction (Algorithm 1). */

static int floor_div2(int e) { return (e >= 0) ? e / 2 : -((-e + 1) / 2); }

/* level_of_detail(|p_cam - x|) = floor(log2 d) with d^2 evaluated in binary32. */
int orc_level_of_detail(const float cam[3], float x, float y, float z)
{
    float dx = cam[0] - x;
    float dy = cam[1] - y;
    float dz = cam[2] - z;
    float d2 = (dx * dx + dy * dy) + dz * dz;
    int l;
    if (d2 == 0.0f) {
        l = ORC_LMIN;                       /* log2(0) = -inf, clamped */
    } else if (isinf(d2)) {
        l = ORC_LMAX;
    } else {
        int e;
        (void)frexpf(d2, &e);               /* d2 = m 2^e, m in [1/2, 1) */
        l = floor_div2(e - 1);              /* floor(log2 d) = floor(floor(log2 d2) / 2) */
    }
    if (l < ORC_LMIN) l = ORC_LMIN;
    if (l > ORC_LMAX) l = ORC_LMAX;
    return l;
}

/* per-axis sign class: 1 positive, 2 negative, 0 zero (either sign) */
static uint32_t normal_class(float c) { return (c > 0.0f) ? 1u : ((c < 0.0f) ? 2u : 0u); }

/* i <- hash(x~, ...): the normal is left out of the home index;
 * f <- hash2(x~, n, ...): 0 is the empty-cell sentinel. */
static void key_hashes(uint64_t k, uint64_t mask, uint32_t *home, uint32_t *fp)
{
    const uint64_t kpos = k & ((1ULL << 56) - 1);   /* position and level only */
    *home = (uint32_t)(orc_fmix64(kpos) & mask);
    const uint32_t f = (uint32_t)(orc_splitmix64(k) >> 32);
    *fp = f ? f : 1u;
}

/*
 * Builds key, fingerprint, home index and flags for n vertices.
 * Flagged vertices get key = fp = home = 0.
 * Optional intermediates (each nullable): lvl[2n] = (l, l'), xj[3n] = x',
 * xq[3n] = x~.
 * level_up > 0 quantises x' at the coarser level l' + level_up instead
 * (x~ = floor(x' / (s * 2^(l' + level_up))), that level in the key): the
 * enclosing voxel of multi-level accumulation (Section 3.3.2); a level above
 * the key's range (15) flags the vertex KEYRANGE.
 */
void orc_build_keys(uint64_t n,
                    const float *px, const float *py, const float *pz,
                    const float *nx, const float *ny, const float *nz,
                    const uint8_t *valid, const float cam[3], float s,
                    uint64_t seed, uint64_t idx_base, uint32_t log2_slots,
                    uint64_t *key, uint32_t *fp, uint32_t *home, uint8_t *flags,
                    int32_t *lvl, float *xj, int32_t *xq, int32_t level_up)
{
    const uint64_t mask = (log2_slots >= 64) ? ~0ULL : ((1ULL << log2_slots) - 1);
    for (uint64_t i = 0; i < n; ++i) {
        float x[3] = { px[i], py[i], pz[i] };
        float nr[3] = { nx[i], ny[i], nz[i] };
        key[i] = 0; fp[i] = 0; home[i] = 0; flags[i] = 0;

        int finite = 1;
        for (int c = 0; c < 3; ++c) finite &= isfinite(x[c]) && isfinite(nr[c]);
        if ((valid && valid[i] == 0) || !finite) { flags[i] = ORC_INVALID; continue; }

        /* l <- level_of_detail(|p_cam - x|) */
        int l = orc_level_of_detail(cam, x[0], x[1], x[2]);

        /* jitter(n): uniform point of the cube [-1/2,1/2)^3 projected onto the
         * tangent plane of n */
        orc_pcg32 g;
        orc_pcg32_seed(&g, seed, idx_base + i);
        float r[3];
        for (int c = 0; c < 3; ++c) r[c] = ldexpf((float)(orc_pcg32_next(&g) >> 8), -24) - 0.5f;
        float t = (r[0] * nr[0] + r[1] * nr[1]) + r[2] * nr[2];
        float j[3];
        for (int c = 0; c < 3; ++c) j[c] = r[c] - t * nr[c];

        /* x' <- x + jitter(n) * s * 2^l */
        float h = ldexpf(s, l);
        float xp[3];
        for (int c = 0; c < 3; ++c) xp[c] = x[c] + j[c] * h;

        /* l' <- level_of_detail(|p_cam - x'|) */
        int lp = orc_level_of_detail(cam, xp[0], xp[1], xp[2]);

        /* x~ <- floor(x' / (s * 2^l')), at l' + level_up for a coarser level */
        const int lq = lp + level_up;
        float hp = ldexpf(s, lq);
        int32_t q[3];
        int inrange = 1;
        for (int c = 0; c < 3; ++c) {
            float f = floorf(xp[c] / hp);
            /* |x~| < 2^16 on both sides: -2^16 would fit the 17-bit field, but
             * no neighbour or child search could then reach that voxel */
            if (!(f > -(float)ORC_QMAX && f < (float)ORC_QMAX)) { inrange = 0; q[c] = 0; }
            else q[c] = (int32_t)f;
        }
        if (lvl) { lvl[2 * i] = l; lvl[2 * i + 1] = lp; }
        if (xj) for (int c = 0; c < 3; ++c) xj[3 * i + c] = xp[c];
        if (xq) for (int c = 0; c < 3; ++c) xq[3 * i + c] = q[c];
        if (!inrange || lq > ORC_LMAX) { flags[i] = ORC_KEYRANGE; continue; }

        /* key: 17 bits per offset coordinate, 5 bits level, 6 bits normal */
        uint32_t code = normal_class(nr[0]) | (normal_class(nr[1]) << 2) | (normal_class(nr[2]) << 4);
        uint64_t k = (uint64_t)(uint32_t)(q[0] + ORC_QMAX)
                   | ((uint64_t)(uint32_t)(q[1] + ORC_QMAX) << 17)
                   | ((uint64_t)(uint32_t)(q[2] + ORC_QMAX) << 34)
                   | ((uint64_t)(uint32_t)(lq - ORC_LMIN) << 51)
                   | ((uint64_t)code << 56);
        key_hashes(k, mask, &home[i], &fp[i]);
        key[i] = k;
    }
}

/* Home index and fingerprint of given keys (for key streams that do not
 * come from positions, such as the table-load sweeps). */
void orc_key_hashes(uint64_t n, const uint64_t *key, uint32_t log2_slots, uint32_t *home, uint32_t *fp)
{
    const uint64_t mask = (1ULL << log2_slots) - 1;
    for (uint64_t i = 0; i < n; ++i) key_hashes(key[i], mask, &home[i], &fp[i]);
}

/* Fixed-point radiance.  Only vertices not yet flagged are examined;
 * non-finite radiance sets INVALID, |r 2^F| >= 2^62 sets RADRANGE. */
void orc_quantize_radiance(uint64_t n, const float *r, const float *g, const float *b,
                           int32_t frac_bits, uint8_t *flags, int64_t *q)
{
    for (uint64_t i = 0; i < n; ++i) {
        const float v[3] = { r[i], g[i], b[i] };
        for (int c = 0; c < 3; ++c) q[3 * i + c] = 0;
        if (flags[i]) continue;
        int finite = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
        if (!finite) { flags[i] = ORC_INVALID; continue; }
        int over = 0;
        float sc[3];
        for (int c = 0; c < 3; ++c) {
            sc[c] = ldexpf(v[c], frac_bits);
            if (!(fabsf(sc[c]) < 4611686018427387904.0f)) over = 1;  /* 2^62 */
        }
        if (over) { flags[i] = ORC_RADRANGE; continue; }
        for (int c = 0; c < 3; ++c) q[3 * i + c] = (int64_t)rintf(sc[c]);  /* round half to even */
    }
}

/* ---------------------------------------------------------------------- */
/* Group-by on the key (Eq. (7) partition, Eq. (8) average with w = 1). */

typedef struct { uint64_t key; uint64_t idx; } orc_pair;

static int cmp_pair(const void *a, const void *b)
{
    const orc_pair *x = (const orc_pair *)a, *y = (const orc_pair *)b;
    if (x->key != y->key) return (x->key < y->key) ? -1 : 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

/*
 * Groups unflagged vertices by key.  Outputs (capacity n each):
 * gkey[G] ascending, gcnt[G], gsum[3G], vgroup[n] (-1 for flagged).
 * Returns G, or -1 if a sum leaves int64.
 */
int64_t orc_group_by(uint64_t n, const uint64_t *key, const uint8_t *flags, const int64_t *q,
                     uint64_t *gkey, uint32_t *gcnt, int64_t *gsum, int64_t *vgroup)
{
    orc_pair *p = (orc_pair *)malloc(sizeof(orc_pair) * (n ? n : 1));
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; ++i) {
        vgroup[i] = -1;
        if (!flags[i]) { p[m].key = key[i]; p[m].idx = i; ++m; }
    }
    qsort(p, m, sizeof(orc_pair), cmp_pair);
    int64_t G = 0;
    uint64_t a = 0;
    while (a < m) {
        uint64_t e = a;
        __int128 acc[3] = { 0, 0, 0 };
        while (e < m && p[e].key == p[a].key) {
            for (int c = 0; c < 3; ++c) acc[c] += q[3 * p[e].idx + c];
            vgroup[p[e].idx] = G;
            ++e;
        }
        for (int c = 0; c < 3; ++c) {
            if (acc[c] > (__int128)INT64_MAX || acc[c] < (__int128)INT64_MIN) { free(p); return -1; }
            gsum[3 * G + c] = (int64_t)acc[c];
        }
        gkey[G] = p[a].key;
        gcnt[G] = (uint32_t)(e - a);
        ++G;
        a = e;
    }
    free(p);
    return G;
}

/* ---------------------------------------------------------------------- */
/* Linear probing (Section 3.2), simulated sequentially on exact keys.
 *
 * Two runs over the G distinct keys in ascending order, each starting at
 * home(key) and stepping by one slot modulo 2^m:
 *   run A: unlimited steps; yields the cluster structure, which is the same
 *          for every insertion order (linear probing without deletions);
 *   run B: at most max_probe slots examined; a key that finds none free is
 *          not placed (its vertices stay unfiltered).
 * Outputs: occupied[2^m] from run B, gslot[G] (run B slot or -1),
 * res[0] = total displacement of run B's placed keys,
 * res[1] = longest cluster of run A (L_max),
 * res[2] = 1 if two distinct keys with equal fingerprints share a cluster of
 *          run A (fingerprint alias), else 0,
 * res[3] = keys run B could not place,
 * res[4 + d] = run B keys placed at displacement d (d >= 64 in bin 64).
 * When L_max <= max_probe and no alias, every insertion order, and a table
 * comparing fingerprints only, give run B's occupancy and displacement.
 */
typedef struct { uint64_t cluster; uint32_t fp; } orc_cf;

static int cmp_cf(const void *a, const void *b)
{
    const orc_cf *x = (const orc_cf *)a, *y = (const orc_cf *)b;
    if (x->cluster != y->cluster) return (x->cluster < y->cluster) ? -1 : 1;
    return (x->fp < y->fp) ? -1 : (x->fp > y->fp);
}

void orc_simulate_table(uint64_t G, const uint64_t *gkey, const uint32_t *gfp, const uint32_t *ghome,
                        uint32_t log2_slots, uint32_t max_probe,
                        uint8_t *occupied, int64_t *gslot, uint64_t *res)
{
    const uint64_t S = 1ULL << log2_slots, mask = S - 1;
    (void)gkey;
    for (int k = 0; k < 4 + 65; ++k) res[k] = 0;

    /* run A */
    int64_t *slotA = (int64_t *)malloc(sizeof(int64_t) * (G ? G : 1));
    int64_t *owner = (int64_t *)malloc(sizeof(int64_t) * S);
    for (uint64_t s = 0; s < S; ++s) owner[s] = -1;
    uint64_t placedA = 0;
    for (uint64_t g = 0; g < G; ++g) {
        slotA[g] = -1;
        if (placedA == S) continue;               /* table full */
        uint64_t s = ghome[g];
        while (owner[s] >= 0) s = (s + 1) & mask;
        owner[s] = (int64_t)g;
        slotA[g] = (int64_t)s;
        ++placedA;
    }
    /* clusters of run A: maximal circular runs of occupied slots */
    uint64_t *cl = (uint64_t *)malloc(sizeof(uint64_t) * S);
    uint64_t lmax = 0;
    if (placedA == S) {
        lmax = S;
        for (uint64_t s = 0; s < S; ++s) cl[s] = 0;
    } else {
        uint64_t start = 0;
        while (owner[start] >= 0) start = (start + 1) & mask;   /* an empty slot */
        uint64_t id = 0, run = 0;
        for (uint64_t k = 1; k <= S; ++k) {
            uint64_t s = (start + k) & mask;
            if (owner[s] >= 0) { cl[s] = id; ++run; if (run > lmax) lmax = run; }
            else { ++id; run = 0; }
        }
    }
    res[1] = lmax;
    /* alias: equal fingerprints inside one cluster */
    orc_cf *cf = (orc_cf *)malloc(sizeof(orc_cf) * (placedA ? placedA : 1));
    uint64_t m = 0;
    for (uint64_t g = 0; g < G; ++g)
        if (slotA[g] >= 0) { cf[m].cluster = cl[slotA[g]]; cf[m].fp = gfp[g]; ++m; }
    qsort(cf, m, sizeof(orc_cf), cmp_cf);
    for (uint64_t k = 1; k < m; ++k)
        if (cf[k].cluster == cf[k - 1].cluster && cf[k].fp == cf[k - 1].fp) res[2] = 1;

    /* run B */
    for (uint64_t s = 0; s < S; ++s) { owner[s] = -1; occupied[s] = 0; }
    for (uint64_t g = 0; g < G; ++g) {
        gslot[g] = -1;
        uint64_t s = ghome[g];
        uint64_t d = 0;
        for (; d < max_probe && d < S; ++d) {
            if (owner[s] < 0) break;
            s = (s + 1) & mask;
        }
        if (d < max_probe && d < S && owner[s] < 0) {
            owner[s] = (int64_t)g;
            occupied[s] = 1;
            gslot[g] = (int64_t)s;
            res[0] += d;
            res[4 + (d < 64 ? d : 64)] += 1;
        } else {
            res[3] += 1;
        }
    }
    free(cf); free(cl); free(owner); free(slotA);
}

/* ---------------------------------------------------------------------- */
/* Lookup: average = sum / counter, one rounding to binary32. */
void orc_average(uint64_t G, const uint32_t *gcnt, const int64_t *gsum, int32_t frac_bits, float *gavg)
{
    for (uint64_t g = 0; g < G; ++g)
        for (int c = 0; c < 3; ++c)
            gavg[3 * g + c] = (float)(ldexp((double)gsum[3 * g + c], -frac_bits) / (double)gcnt[g]);
}

/* Per-vertex output: the group's value, or the vertex's own contribution
 * when the vertex is flagged or its group could not be placed. */
void orc_query(uint64_t n, const int64_t *vgroup, const int64_t *gslot, const float *gval,
               const uint32_t *gcnt, const float *r, const float *g, const float *b,
               float *out, uint32_t *cnt_out, uint8_t *flags)
{
    for (uint64_t i = 0; i < n; ++i) {
        int64_t k = vgroup[i];
        if (k >= 0 && gslot && gslot[k] < 0) { flags[i] |= ORC_OVERFLOW; k = -1; }
        if (k < 0) {
            out[3 * i] = r[i]; out[3 * i + 1] = g[i]; out[3 * i + 2] = b[i];
            cnt_out[i] = 0;
        } else {
            for (int c = 0; c < 3; ++c) out[3 * i + c] = gval[3 * k + c];
            cnt_out[i] = gcnt[k];
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Exponential moving average over two sets of averages (Section 3.4.1):
 * c = alpha * c_old + (1 - alpha) * c_new for keys present in the previous
 * set, c = c_new otherwise.  pkey must be ascending. */
void orc_temporal_ema(uint64_t G, const uint64_t *gkey, const float *gnew,
                      uint64_t Gp, const uint64_t *pkey, const float *pold,
                      float alpha_old, float *out)
{
    const float beta = 1.0f - alpha_old;
    for (uint64_t g = 0; g < G; ++g) {
        /* binary search for the key in the previous set */
        uint64_t lo = 0, hi = Gp;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (pkey[mid] < gkey[g]) lo = mid + 1; else hi = mid;
        }
        int found = (lo < Gp && pkey[lo] == gkey[g]);
        for (int c = 0; c < 3; ++c) {
            if (found) {
                float a = alpha_old * pold[3 * lo + c];
                float b = beta * gnew[3 * g + c];
                out[3 * g + c] = a + b;
            } else {
                out[3 * g + c] = gnew[3 * g + c];
            }
        }
    }
}

/* Temporal integration (Section 3.4.1): with alpha = N_old / (N_old + N_new)
 * the blend of the previous value (N_old samples) and this frame's average
 * (N_new samples) is their pooled mean.  The threshold heuristic of the same
 * section keeps the stored count at most max_samples, after which the
 * history keeps that weight.  alpha is the binary32 quotient of the two
 * counts (exact integers below 2^24), then c = alpha*c_old + (1-alpha)*c_new
 * with each product and the sum rounded, as for the moving average. */
void orc_temporal_integrate(uint64_t G, const uint64_t *gkey, const float *gnew, const uint32_t *gcnt,
                            uint64_t Gp, const uint64_t *pkey, const float *pold, const uint32_t *pcnt,
                            uint32_t max_samples, float *out, uint32_t *outn)
{
    for (uint64_t g = 0; g < G; ++g) {
        uint64_t lo = 0, hi = Gp;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (pkey[mid] < gkey[g]) lo = mid + 1; else hi = mid;
        }
        int found = (lo < Gp && pkey[lo] == gkey[g]);
        uint64_t n = gcnt[g];
        if (found) {
            const uint64_t nsum = (uint64_t)pcnt[lo] + gcnt[g];
            const float alpha = (float)pcnt[lo] / (float)nsum;
            const float beta = 1.0f - alpha;
            for (int c = 0; c < 3; ++c) {
                float a = alpha * pold[3 * lo + c];
                float b = beta * gnew[3 * g + c];
                out[3 * g + c] = a + b;
            }
            n = nsum;
        } else {
            for (int c = 0; c < 3; ++c) out[3 * g + c] = gnew[3 * g + c];
        }
        outn[g] = (uint32_t)(n < max_samples ? n : max_samples);
    }
}

/* ---------------------------------------------------------------------- */
/* Fallbacks for voxels with few vertices (Section 3.3).  A placed voxel
 * whose count is below `below` takes the pooled average of a set of placed
 * voxels around it: the integer sums and counts of the set are added and
 * divided once, as for a single voxel.
 *   mode 0, neighbourhood search: the 3 x 3 x 3 block of voxels at the
 *     same level of detail and normal class whose quantised coordinates
 *     differ from its own by at most one per axis (itself included;
 *     coordinates outside the key range are skipped);
 *   mode 1, similar normals along the probe run: the voxels with its
 *     position and level whose normal class vector (one of -1, 0, +1 per
 *     axis) has a positive dot product with its own -- the fingerprint sees
 *     the normal but the home index does not, so these voxels share its
 *     home slot and probe run.
 * gval is overwritten for the pooled voxels, which are marked in gpooled.
 * gkey must be ascending.  Returns -1 if a pooled sum leaves int64. */
static int64_t find_key(uint64_t G, const uint64_t *gkey, uint64_t k)
{
    uint64_t lo = 0, hi = G;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (gkey[mid] < k) lo = mid + 1; else hi = mid;
    }
    return (lo < G && gkey[lo] == k) ? (int64_t)lo : -1;
}

static int class_sign(uint64_t code, int axis)
{
    const uint64_t v = (code >> (2 * axis)) & 3u;
    return v == 1 ? 1 : (v == 2 ? -1 : 0);
}

int orc_low_density(uint64_t G, const uint64_t *gkey, const uint32_t *gcnt, const int64_t *gsum,
                    const uint8_t *placed, uint32_t below, int mode, int32_t frac_bits,
                    float *gval, uint8_t *gpooled)
{
    const uint64_t coord_mask = (1ull << 51) - 1;   /* the three 17-bit coordinates */
    const uint64_t pos_mask = (1ull << 56) - 1;     /* coordinates and level */
    for (uint64_t g = 0; g < G; ++g) {
        gpooled[g] = 0;
        if (!placed[g] || gcnt[g] >= below) continue;
        const uint64_t K = gkey[g];
        uint64_t cand[27];
        int nc = 0;
        if (mode == 0) {
            int x[3];
            for (int c = 0; c < 3; ++c) x[c] = (int)((K >> (17 * c)) & 0x1ffffu) - 65536;
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        const int y[3] = {x[0] + dx, x[1] + dy, x[2] + dz};
                        int ok = 1;
                        for (int c = 0; c < 3; ++c) ok = ok && y[c] > -65536 && y[c] < 65536;
                        if (!ok) continue;
                        cand[nc++] = (K & ~coord_mask) | (uint64_t)(y[0] + 65536) |
                                     ((uint64_t)(y[1] + 65536) << 17) | ((uint64_t)(y[2] + 65536) << 34);
                    }
        } else {
            const uint64_t code = K >> 56;
            for (uint64_t cx = 0; cx < 3; ++cx)
                for (uint64_t cy = 0; cy < 3; ++cy)
                    for (uint64_t cz = 0; cz < 3; ++cz) {
                        const uint64_t other = cx | (cy << 2) | (cz << 4);
                        int dot = 0;
                        for (int c = 0; c < 3; ++c) dot += class_sign(code, c) * class_sign(other, c);
                        if (dot > 0) cand[nc++] = (K & pos_mask) | (other << 56);
                    }
        }
        __int128 S[3] = {0, 0, 0};
        uint64_t N = 0;
        for (int k = 0; k < nc; ++k) {
            const int64_t j = find_key(G, gkey, cand[k]);
            if (j < 0 || !placed[j]) continue;
            N += gcnt[j];
            for (int c = 0; c < 3; ++c) S[c] += gsum[3 * j + c];
        }
        for (int c = 0; c < 3; ++c) {
            if (S[c] > (__int128)INT64_MAX || S[c] < (__int128)INT64_MIN) return -1;
            gval[3 * g + c] = (float)(ldexp((double)(int64_t)S[c], -frac_bits) / (double)N);
        }
        gpooled[g] = 1;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* A history of voxel values kept beyond the previous frame, with eviction
 * by priority (Section 3.4.3).  Direct-mapped: the voxel with key K lives
 * only in slot fmix64(K) mod 2^h.  Each slot holds a 64-bit word, the key,
 * the value (c, N) and the frame it was last written (stamp); an empty slot
 * has word = all ones.  The word's top byte is a priority, its low 56 bits a
 * hash of the key (SplitMix64(K) mod 2^56), so that of all voxels competing
 * for a slot the one with the smallest word stays: a single minimum decides
 * collisions and eviction.  Priority (smaller = kept):
 *   (min(age, 15) << 4) | (15 - min(floor(log2 N), 15)),
 * age = frames since the voxel was written: recent voxels first, then those
 * with more samples.
 * One frame:
 *   1. orc_history_lookup: hit[g] = 1 and old[g] = the slot's (c, N) when the
 *      slot of gkey[g] is occupied by that key; the frame's values are then
 *      blended against old with the arithmetic used for the previous
 *      frame's set;
 *   2. orc_history_update, given the frame's blended values gval [G,3] and
 *      counts gn [G]: every occupied slot whose age = frame - stamp exceeds
 *      max_age is emptied and the others get their word recomputed with
 *      their age; then the frame's voxels compete: a slot keeps the minimum
 *      of its word and the words (age 0) of the voxels mapped to it, and a
 *      voxel whose word is that minimum writes its key, value and
 *      stamp = frame. */
static uint32_t floor_log2_u32(uint32_t x) { uint32_t r = 0; while (x >>= 1) ++r; return r; }

static uint64_t history_word(uint64_t key, uint32_t age, uint32_t count)
{
    const uint32_t a = age < 15 ? age : 15;
    const uint32_t lg = floor_log2_u32(count ? count : 1);
    const uint32_t p = (a << 4) | (15 - (lg < 15 ? lg : 15));
    return ((uint64_t)p << 56) | (orc_splitmix64(key) & ((1ull << 56) - 1));
}

void orc_history_lookup(uint64_t G, const uint64_t *gkey, uint32_t log2_hist, const uint64_t *hword,
                        const uint64_t *hkey, const float *hval, uint8_t *hit, float *old)
{
    const uint64_t mask = (1ull << log2_hist) - 1;
    for (uint64_t g = 0; g < G; ++g) {
        const uint64_t s = orc_fmix64(gkey[g]) & mask;
        hit[g] = (hword[s] != ~0ull && hkey[s] == gkey[g]);
        for (int c = 0; c < 4; ++c) old[4 * g + c] = hit[g] ? hval[4 * s + c] : 0.0f;
    }
}

void orc_history_update(uint64_t G, const uint64_t *gkey, const float *gval, const uint32_t *gn,
                        uint32_t log2_hist, uint32_t max_age, uint32_t frame,
                        uint64_t *hword, uint64_t *hkey, float *hval, uint32_t *hstamp)
{
    const uint64_t mask = (1ull << log2_hist) - 1;
    for (uint64_t s = 0; s <= mask; ++s) {
        if (hword[s] == ~0ull) continue;
        const uint32_t age = frame - hstamp[s];
        if (age > max_age) hword[s] = ~0ull;
        else hword[s] = history_word(hkey[s], age, (uint32_t)hval[4 * s + 3]);
    }
    for (uint64_t g = 0; g < G; ++g) {
        const uint64_t s = orc_fmix64(gkey[g]) & mask;
        const uint64_t w = history_word(gkey[g], 0, gn[g]);
        if (w < hword[s]) hword[s] = w;
    }
    for (uint64_t g = 0; g < G; ++g) {
        const uint64_t s = orc_fmix64(gkey[g]) & mask;
        if (hword[s] != history_word(gkey[g], 0, gn[g])) continue;
        hkey[s] = gkey[g];
        for (int c = 0; c < 3; ++c) hval[4 * s + c] = gval[3 * g + c];
        hval[4 * s + 3] = (float)gn[g];
        hstamp[s] = frame;
    }
}

/* ---------------------------------------------------------------------- */
/* Pixel resolve (Section 3): after filtering, each selected vertex's value
 * is multiplied by its throughput (the attenuation from the camera along its
 * path up to the vertex) and accumulated in its pixel.  Vertices are stored
 * bounce-major: vertex b of pixel p is at b * pixels + p.  Per pixel and
 * channel, in binary32 with each product and sum rounded, over b = 0, 1, ...:
 * acc = acc + t * c for the vertices with valid != 0 (valid NULL: all);
 * t = 1 when throughput is NULL.  accumulate != 0 starts from the pixel's
 * value, else from 0. */
void orc_resolve_pixels(uint64_t pixels, uint32_t verts_per_path, const float *c3, const float *t3,
                        const uint8_t *valid, int accumulate, float *px3)
{
    for (uint64_t p = 0; p < pixels; ++p) {
        for (int ch = 0; ch < 3; ++ch) {
            float acc = accumulate ? px3[3 * p + ch] : 0.0f;
            for (uint32_t b = 0; b < verts_per_path; ++b) {
                const uint64_t v = (uint64_t)b * pixels + p;
                if (valid && valid[v] == 0) continue;
                const float t = t3 ? t3[3 * v + ch] : 1.0f;
                const float prod = t * c3[3 * v + ch];
                acc = acc + prod;
            }
            px3[3 * p + ch] = acc;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Changes of resolution across frames (Section 3.4.2).  A voxel of this
 * frame whose key is absent from the previous set may find its region there
 * one level coarser or finer:
 *   coarser (the resolution increased): the parent voxel, level l' + 1 and
 *     cell coordinates floor-divided by 2, its value distributed to the
 *     finer voxel: c_old = the parent's value, N_old = floor(N_parent / 8)
 *     (its samples spread over its 8 children; with N_old = 0 in
 *     integration the parent is not used);
 *   finer (the resolution decreased): the 8 children, level l' - 1 and cell
 *     coordinates 2x~ + (0 or 1) per axis, added up: N_old = sum of their
 *     counts, c_old = (float)(sum_j N_j c_j / N_old) accumulated in double in
 *     the order j = dx + 2 dy + 4 dz.
 * The exact key comes first, then the parent, then the children; the blend
 * (mode 0 moving average with alpha_old, mode 1 integration with
 * max_samples) is the arithmetic of orc_temporal_ema / orc_temporal_integrate.
 * how[g]: 0 not found, 1 exact, 2 parent, 3 children.  pkey ascending. */
static int64_t find_prev(uint64_t Gp, const uint64_t *pkey, uint64_t k)
{
    uint64_t lo = 0, hi = Gp;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (pkey[mid] < k) lo = mid + 1; else hi = mid;
    }
    return (lo < Gp && pkey[lo] == k) ? (int64_t)lo : -1;
}

void orc_temporal_levels(uint64_t G, const uint64_t *gkey, const float *gnew, const uint32_t *gcnt,
                         uint64_t Gp, const uint64_t *pkey, const float *pold, const uint32_t *pcnt,
                         int mode, float alpha_old, uint32_t max_samples, float *out, uint32_t *outn,
                         uint8_t *how)
{
    for (uint64_t g = 0; g < G; ++g) {
        const uint64_t K = gkey[g];
        int x[3];
        for (int c = 0; c < 3; ++c) x[c] = (int)((K >> (17 * c)) & 0x1ffffu) - 65536;
        const int lp = (int)((K >> 51) & 31u) - 16;
        const uint64_t code = K >> 56;
        float cold[3] = {0, 0, 0};
        uint64_t nold = 0;
        how[g] = 0;
        int64_t j = find_prev(Gp, pkey, K);
        if (j >= 0) {
            how[g] = 1;
            for (int c = 0; c < 3; ++c) cold[c] = pold[3 * j + c];
            nold = pcnt[j];
        }
        if (!how[g] && lp + 1 <= ORC_LMAX) {
            uint64_t P = (code << 56) | ((uint64_t)(lp + 1 - ORC_LMIN) << 51);
            for (int c = 0; c < 3; ++c) P |= (uint64_t)(uint32_t)((x[c] >> 1) + 65536) << (17 * c);
            j = find_prev(Gp, pkey, P);
            if (j >= 0 && (mode == 0 || pcnt[j] / 8 >= 1)) {
                how[g] = 2;
                for (int c = 0; c < 3; ++c) cold[c] = pold[3 * j + c];
                nold = pcnt[j] / 8;
            }
        }
        if (!how[g] && lp - 1 >= ORC_LMIN) {
            double acc[3] = {0, 0, 0};
            uint64_t n = 0;
            for (int d = 0; d < 8; ++d) {
                uint64_t C = (code << 56) | ((uint64_t)(lp - 1 - ORC_LMIN) << 51);
                int ok = 1;
                for (int c = 0; c < 3; ++c) {
                    const int y = 2 * x[c] + ((d >> c) & 1);
                    ok = ok && y > -65536 && y < 65536;
                    C |= (uint64_t)(uint32_t)(y + 65536) << (17 * c);
                }
                if (!ok) continue;
                j = find_prev(Gp, pkey, C);
                if (j < 0) continue;
                n += pcnt[j];
                for (int c = 0; c < 3; ++c) acc[c] += (double)pcnt[j] * (double)pold[3 * j + c];
            }
            if (n) {
                how[g] = 3;
                for (int c = 0; c < 3; ++c) cold[c] = (float)(acc[c] / (double)n);
                nold = n;
            }
        }
        uint64_t nkeep = gcnt[g];
        if (!how[g]) {
            for (int c = 0; c < 3; ++c) out[3 * g + c] = gnew[3 * g + c];
        } else {
            float alpha = alpha_old;
            if (mode == 1) {
                const uint64_t nsum = nold + gcnt[g];
                alpha = (float)nold / (float)nsum;
                nkeep = nsum;
            }
            const float beta = 1.0f - alpha;
            for (int c = 0; c < 3; ++c) {
                const float a = alpha * cold[c];
                const float b = beta * gnew[3 * g + c];
                out[3 * g + c] = a + b;
            }
        }
        outn[g] = (uint32_t)(mode == 1 ? (nkeep < max_samples ? nkeep : max_samples) : gcnt[g]);
    }
}
