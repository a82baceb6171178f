// Learned fallback for sparse cells on gfx950: selection of training and
// sparse vertices, a fused BF16 MFMA training step (features, forward,
// backward, per-workgroup gradient sums), a deterministic gradient reduction
// with Adam, and inference.  MFMA: v_mfma_f32_16x16x16_bf16 (wave64), with
//   A operand: lane l holds A[l % 16][4 (l / 16) + 0..3]
//   B operand: lane l holds B[4 (l / 16) + 0..3][l % 16]
//   C/D:       lane l holds D[4 (l / 16) + 0..3][l % 16].
#include "pf_device.h"
#include "pf_kernels.h"

namespace pfk {

namespace mlp {

constexpr int kIn = PF_MLP_IN;       // 80
constexpr int kH = PF_MLP_HIDDEN;    // 64
constexpr int kOutPad = 16;
constexpr int kOut = 3;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kIn;       // 5120
constexpr int kOffW2 = kOffB1 + kH;             // 5184
constexpr int kOffB2 = kOffW2 + kH * kH;        // 9280
constexpr int kOffW3 = kOffB2 + kH;             // 9344
constexpr int kOffB3 = kOffW3 + kOutPad * kH;   // 10368
constexpr int kNParam = kOffB3 + kOutPad;       // 10384
static_assert(kNParam == PF_MLP_NPARAM, "parameter packing");
constexpr int kBS = PF_MLP_BLOCK_SAMPLES;      // 64 samples per workgroup (4 waves x 16)
// LDS row strides of the arrays whose rows hold 64 values: 72 elements (144
// bytes), so that the 16 rows a wavefront's MFMA operand loads and
// transposed stores touch fall on different banks (a 128-byte stride puts
// them all on two)
constexpr int kLdIn = kIn + 8; // rows of W1 (80 inputs in slot order)
constexpr int kLdH = kH + 8;   // rows of 64 hidden units (weights W2, W3, W2^T; activations)
constexpr int kLdS = kBS + 8;  // rows of 64 samples (transposed operands)
constexpr int kThreads = 256;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// float -> bfloat16, round to nearest even, NaN kept quiet; a select, not a
// branch (the conversions sit between the products of every layer)
__device__ __forceinline__ uint16_t bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint32_t rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const uint32_t quiet = (u >> 16) | 0x40u;
    return (uint16_t)(((u & 0x7fffffffu) > 0x7f800000u) ? quiet : rounded);
}

// Waits for this wave's LDS operations only (lgkmcnt 0, vmcnt and expcnt at
// their maxima), before a wave barrier that publishes LDS stores to the other
// lanes; global loads issued ahead stay in flight.
__device__ __forceinline__ void lds_wait() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Two floats -> two bfloat16 (low, high half) with gfx950's conversion
// instruction: round to nearest even, identical to bf16() for every value
// but FP32 denormals, which it flushes to zero.  Used where a denormal
// cannot occur (the positional features) or would not matter (activations
// and gradients inside the products); the weights' BF16 copy and the
// normal and view-direction features keep bf16().
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16x2(float lo, float hi) {
    const f32x2_t v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

__device__ __forceinline__ v4s ld4(const uint16_t *p) { return *reinterpret_cast<const v4s *>(p); }

__device__ __forceinline__ void st4(uint16_t *p, float a, float b, float c, float d) {
    const uint2 v = {bf16x2(a, b), bf16x2(c, d)};
    *reinterpret_cast<uint2 *>(p) = v;
}

// FP64 -> FP32 -> BF16, zeros as +0 (sinpi and cospi may return -0)
__device__ __forceinline__ uint16_t to_feature(double v) {
    v = v + 0.0;
    return bf16((float)v);
}

// sin(pi t) and cos(pi t) in FP32 for the dyadic phase t = m 2^e (m odd,
// |m| < 2^17, e <= 15).  Every step of the reduction is exact: t itself
// (with e clamped to 1: every even integer phase gives 0 and 1, as 2 does),
// 2t, its nearest integer k, and r = t - k/2 with |r| <= 1/4 (a multiple of
// 2^e with at most 18 significant bits).  sin(pi r) and cos(pi r) come from
// their Taylor series (through r^9 and r^10, truncation below 2^-28
// relative at |r| = 1/4), coefficients rounded to FP32 and evaluated with
// explicit fused multiply-adds; each value lies within 3 FP32 ulps of the
// true one (2 observed over every phase), and the quadrant k mod 4 swaps
// and negates them exactly.  Returns true when either value lies within
// kTieGuard bit patterns of a BF16 rounding midpoint: only there could the
// FP64 value, rounded FP64 -> FP32 -> BF16, round to a different BF16 than
// this FP32 value does (never for an integer phase, whose values are exact).
constexpr uint32_t kTieGuard = 16;
__device__ __forceinline__ bool near_bf16_tie(float y) {
    const uint32_t lo = __float_as_uint(y) & 0xffffu;
    return lo - (0x8000u - kTieGuard) <= 2u * kTieGuard;
}
__device__ __forceinline__ bool dyadic_sincospi(int32_t m, int e, float &so, float &co) {
    const float t = ldexpf((float)m, e < 1 ? e : 1);
    const float k = __builtin_rintf(2.0f * t);  // nearest multiple of 1/2, ties to even
    const float r = fmaf(k, -0.5f, t);
    const int kq = (int)k;
    const float r2 = r * r;
    float p = fmaf(r2, 0x1.507834p-4f, -0x1.32d2ccp-1f);  // pi^9/9!, -pi^7/7!
    p = fmaf(r2, p, 0x1.466bc6p+1f);                      // pi^5/5!
    p = fmaf(r2, p, -0x1.4abbcep+2f);                     // -pi^3/3!
    p = fmaf(r2, p, 0x1.921fb6p+1f);                      // pi
    const float sr = r * p;
    float c = fmaf(r2, -0x1.a6d1f2p-6f, 0x1.e1f506p-3f);  // -pi^10/10!, pi^8/8!
    c = fmaf(r2, c, -0x1.55d3c8p+0f);                     // -pi^6/6!
    c = fmaf(r2, c, 0x1.03c1f0p+2f);                      // pi^4/4!
    c = fmaf(r2, c, -0x1.3bd3ccp+2f);                     // -pi^2/2!
    const float cr = fmaf(r2, c, 1.0f);
    const bool odd = (kq & 1) != 0, neg_s = (kq & 2) != 0, neg_c = ((kq + 1) & 2) != 0;
    const float sv = odd ? cr : sr, cv = odd ? sr : cr;
    so = (neg_s ? -sv : sv) + 0.0f;  // zeros as +0
    co = (neg_c ? -cv : cv) + 0.0f;
    return near_bf16_tie(so) || near_bf16_tie(co);
}

// Positional-encoding pair j of coordinate c: sin and cos of pi t with the
// exact phase t = (q + 1/2) 2^(lp - 10 + j) = (2q + 1) 2^e, e = lp - 11 + j,
// from dyadic_sincospi, or, near a BF16 rounding midpoint, from one FP64
// sincospi, so that both are the FP64 values rounded FP64 -> FP32 -> BF16.
// No other branch: the lanes of a wavefront hold vertices of different
// levels.  FP32 -> BF16 of both values is one conversion instruction: the
// values are 0, +-1 or at least sin(pi 2^-27) in magnitude (the phase is an
// odd multiple of 2^e, e >= -27, so it is never within 2^-27 of an
// integer), never an FP32 denormal.
__device__ __forceinline__ void pe_pair(int32_t qc, int lp, int j, uint16_t &sv, uint16_t &cv) {
    float sn, cs;
    if (dyadic_sincospi(2 * qc + 1, lp - 11 + j, sn, cs)) {
        double s64, c64;
        sincospi(ldexp((double)qc + 0.5, lp - 10 + j), &s64, &c64);  // exact phase
        sn = (float)(s64 + 0.0);
        cs = (float)(c64 + 0.0);
    }
    const uint32_t both = bf16x2(sn, cs);
    sv = (uint16_t)both;
    cv = (uint16_t)(both >> 16);
}

// Feature f of a vertex (f in [0, 80)), FP64 then FP64 -> FP32 -> BF16, zeros as +0.
__device__ __forceinline__ uint16_t feature(int f, const int32_t q[3], int lp, const float x[3], const float n[3],
                                            const float cam[3]) {
    double v = 0.0;
    if (f < 72) {
        const int j = f / 6, r = f % 6, c = r % 3;
        uint16_t sv, cv;
        pe_pair(q[c], lp, j, sv, cv);
        return r < 3 ? sv : cv;
    } else if (f < 75) {
        v = (double)n[f - 72];
    } else if (f < 78) {
        const double dx = (double)x[0] - (double)cam[0];
        const double dy = (double)x[1] - (double)cam[1];
        const double dz = (double)x[2] - (double)cam[2];
        const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
        const double len = sqrt((xx + yy) + zz);
        const double d[3] = {dx, dy, dz};
        v = d[f - 75] / len;
    }
    return to_feature(v);
}

// The 80 inputs of a vertex are computed by its 4 lanes lg = 0..3 (16
// vertices a wave, lane = 16 lg + vertex), 20 values each: lane lg's m-th
// value is the sine (m even) or cosine (m odd) of positional pair
// lg + 4 (m / 2) for m < 18, input 72 + lg for m = 18 and input 76 + lg for
// m = 19.  Inference keeps them in slot order, lane lg's m-th value in slot
// 16 (m / 4) + 4 lg + m % 4, which is the layout of a 16 x 16 x 16
// product's operand with the vertices along its 16 columns (its W1 columns
// are permuted to match when staged); training stores them in input order.
__device__ __forceinline__ int slot_of_input(int f) {
    if (f >= 72) return 64 + 4 * ((f - 72) & 3) + 2 + ((f - 72) >> 2);
    const int j = f / 6, r = f % 6, p = 3 * j + r % 3, m = 2 * (p >> 2) + r / 3;
    return 16 * (m >> 2) + 4 * (p & 3) + (m & 3);
}
// input index of lane group lg's m-th value
__device__ __forceinline__ int input_of_lane_value(int lg, int m) {
    if (m >= 18) return (m == 18 ? 72 : 76) + lg;
    const int p = lg + 4 * (m >> 1), j = p / 3, c = p % 3;
    return 6 * j + 3 * (m & 1) + c;
}

// The 20 values of lane group lg of one vertex, in slot order:
// put(m, value) for m = 0..19 (m known at compile time once unrolled).
template <typename Put>
__device__ __forceinline__ void vertex_slots(int lg, const int32_t q[3], int lp, const float x[3], const float n[3],
                                             const float cam[3], Put put) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {  // independent phases: unrolled so that their FP64 chains interleave
        const int pi = lg + 4 * k, j = pi / 3, c = pi % 3;
        const int32_t qc = c == 0 ? q[0] : (c == 1 ? q[1] : q[2]);  // selects: q stays in registers
        uint16_t sv, cv;
        pe_pair(qc, lp, j, sv, cv);
        put(2 * k, sv);
        put(2 * k + 1, cv);
    }
    // inputs 72 + lg and 76 + lg: the normal (72..74), the view direction
    // (75..77) and two zeros (78, 79); a lane needs at most one component of
    // the direction, so it divides once
    const double dx = (double)x[0] - (double)cam[0];
    const double dy = (double)x[1] - (double)cam[1];
    const double dz = (double)x[2] - (double)cam[2];
    const double len = sqrt((dx * dx + dy * dy) + dz * dz);
    const double dir = (lg == 3 ? dx : (lg == 0 ? dy : dz)) / len;
    const float nl = lg == 0 ? n[0] : (lg == 1 ? n[1] : n[2]);
    put(18, to_feature(lg < 3 ? (double)nl : dir));
    put(19, to_feature(lg < 2 ? dir : 0.0));
}

struct Geo {
    const uint64_t *key;
    const float *px, *py, *pz, *nx, *ny, *nz;
    float cam[3];
};

__device__ __forceinline__ void vertex_inputs(const Geo &g, uint32_t v, int32_t q[3], int &lp, float x[3],
                                              float n[3]) {
    const uint64_t k = g.key[v];
    q[0] = (int32_t)((k >> 0) & 0x1ffffu) - 65536;
    q[1] = (int32_t)((k >> 17) & 0x1ffffu) - 65536;
    q[2] = (int32_t)((k >> 34) & 0x1ffffu) - 65536;
    lp = (int)((k >> 51) & 31u) - 16;
    x[0] = g.px[v];
    x[1] = g.py[v];
    x[2] = g.pz[v];
    n[0] = g.nx[v];
    n[1] = g.ny[v];
    n[2] = g.nz[v];
}

// Stages the BF16 weights and the FP32 biases in LDS (and, for training,
// the transposes the backward pass reads).
struct Weights {
    uint16_t w1[kH * kLdIn];  // columns in input order (training) or slot order (inference)
    uint16_t w2[kH * kLdH];
    uint16_t w3[kOutPad * kLdH];
    float b1[kH], b2[kH], b3[kOutPad];
};

struct WeightsT {
    uint16_t w2t[kH * kLdH];
    uint16_t w3t[kH * kOutPad];
};

// The weights' global loads, all issued before any is stored (16-byte loads
// of the BF16 copy; wb is 16-byte aligned and every matrix starts and every
// row ends on a 16-byte boundary), held in registers until stage().
template <int NT>
struct WeightLoadsT {
    static constexpr int kW1 = kH * kIn / 8, kW2 = kH * kH / 8, kW3 = kOutPad * kH / 8, kB = kH + kH + kOutPad;
    static constexpr int kN1 = (kW1 + NT - 1) / NT, kN2 = (kW2 + NT - 1) / NT;
    uint4 w1[kN1], w2[kN2], w3;
    float b;

    __device__ __forceinline__ void issue(const uint16_t *wb, const float *w) {
        const uint4 *v1 = reinterpret_cast<const uint4 *>(wb + kOffW1);
        const uint4 *v2 = reinterpret_cast<const uint4 *>(wb + kOffW2);
        const uint4 *v3 = reinterpret_cast<const uint4 *>(wb + kOffW3);
        // unconditional loads of clamped indices (a guarded load becomes a
        // branch that waits for it); stage() stores only the valid ones
        const int t = threadIdx.x;
#pragma unroll
        for (int k = 0; k < kN1; ++k) w1[k] = v1[min(t + k * NT, kW1 - 1)];
#pragma unroll
        for (int k = 0; k < kN2; ++k) w2[k] = v2[min(t + k * NT, kW2 - 1)];
        w3 = v3[min(t, kW3 - 1)];
        const int tb = min(t, kB - 1);
        b = w[tb < kH ? kOffB1 + tb : (tb < 2 * kH ? kOffB2 + tb - kH : kOffB3 + tb - 2 * kH)];
    }

    // element j of 8 BF16 values (by shifts: taking the address of the
    // registers would move them to scratch memory)
    static __device__ __forceinline__ uint16_t half(const uint4 &u, int j) {
        const uint32_t word = (j >> 1) == 0 ? u.x : (j >> 1) == 1 ? u.y : (j >> 1) == 2 ? u.z : u.w;
        return (uint16_t)((j & 1) ? word >> 16 : word & 0xffffu);
    }

    // Stores the BF16 weights (row-padded W2, W3), the FP32 biases and, for
    // training, the transposes the backward pass reads.  Unconditional, like
    // the loads: a lane past the end stores the clamped last element again
    // (the same value to the same address), so no branch holds a load back.
    template <bool kSlotOrder>
    __device__ __forceinline__ void stage(Weights &W, WeightsT *T) const {
        const int t = threadIdx.x;
#pragma unroll
        for (int k = 0; k < kN1; ++k) {
            const int e = 8 * min(t + k * NT, kW1 - 1), row = e / kIn, f0 = e % kIn;
            if (kSlotOrder) {
#pragma unroll
                for (int j = 0; j < 8; ++j) W.w1[row * kLdIn + slot_of_input(f0 + j)] = half(w1[k], j);
            } else {
                *reinterpret_cast<uint4 *>(W.w1 + row * kLdIn + f0) = w1[k];
            }
        }
#pragma unroll
        for (int k = 0; k < kN2; ++k) {
            const int i = min(t + k * NT, kW2 - 1);
            const int row = (8 * i) / kH, col = (8 * i) % kH;
            *reinterpret_cast<uint4 *>(W.w2 + row * kLdH + col) = w2[k];
            if (T) {
#pragma unroll
                for (int j = 0; j < 8; ++j) T->w2t[(col + j) * kLdH + row] = half(w2[k], j);
            }
        }
        {
            const int i = min(t, kW3 - 1);
            const int row = (8 * i) / kH, col = (8 * i) % kH;
            *reinterpret_cast<uint4 *>(W.w3 + row * kLdH + col) = w3;
            if (T) {
#pragma unroll
                for (int j = 0; j < 8; ++j) T->w3t[(col + j) * kOutPad + row] = half(w3, j);
            }
        }
        const int tb = min(t, kB - 1);
        float *bias = tb < kH ? W.b1 + tb : (tb < 2 * kH ? W.b2 + tb - kH : W.b3 + tb - 2 * kH);
        *bias = b;
    }
};

using WeightLoads = WeightLoadsT<kThreads>;

// Forward pass of one wave's 16-row tile (rows r0..r0+15 of x, a1, a2 with
// row strides kIn / lda).  Keeps z1, z2 (C layout) for the backward pass and
// returns y (C layout, columns = outputs).  If a1t/a2t are given, the
// transposed activations are stored too (row stride ldt).
__device__ __forceinline__ v4f forward_tile(const Weights &W, const uint16_t *x, uint16_t *a1, uint16_t *a2, int lda,
                                            uint16_t *a1t, uint16_t *a2t, int ldt, int r0, v4f z1[4], v4f z2[4]) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    // layer 1
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) z1[nt] = v4f{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < kIn / 16; ++kk) {
        const v4s a = ld4(x + (r0 + lr) * kIn + kk * 16 + 4 * lg);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) z1[nt] = mfma(a, ld4(W.w1 + (nt * 16 + lr) * kLdIn + kk * 16 + 4 * lg), z1[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int n = nt * 16 + lr;
        float h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            z1[nt][i] += W.b1[n];
            h[i] = z1[nt][i] > 0.0f ? z1[nt][i] : 0.0f;
            a1[(r0 + 4 * lg + i) * lda + n] = (uint16_t)bf16x2(h[i], 0.0f);
        }
        if (a1t) st4(a1t + n * ldt + r0 + 4 * lg, h[0], h[1], h[2], h[3]);
    }
    lds_wait();
    __builtin_amdgcn_wave_barrier();
    // layer 2
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) z2[nt] = v4f{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < kH / 16; ++kk) {
        const v4s a = ld4(a1 + (r0 + lr) * lda + kk * 16 + 4 * lg);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) z2[nt] = mfma(a, ld4(W.w2 + (nt * 16 + lr) * kLdH + kk * 16 + 4 * lg), z2[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int n = nt * 16 + lr;
        float h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            z2[nt][i] += W.b2[n];
            h[i] = z2[nt][i] > 0.0f ? z2[nt][i] : 0.0f;
            a2[(r0 + 4 * lg + i) * lda + n] = (uint16_t)bf16x2(h[i], 0.0f);
        }
        if (a2t) st4(a2t + n * ldt + r0 + 4 * lg, h[0], h[1], h[2], h[3]);
    }
    lds_wait();
    __builtin_amdgcn_wave_barrier();
    // layer 3 (16 padded outputs)
    v4f y = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < kH / 16; ++kk)
        y = mfma(ld4(a2 + (r0 + lr) * lda + kk * 16 + 4 * lg), ld4(W.w3 + lr * kLdH + kk * 16 + 4 * lg), y);
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] += W.b3[lr];
    return y;
}

// Sum over the 4 lane groups (rows 4g..4g+3) of a per-lane value: the wave's
// total for column lane % 16, in a fixed order.
__device__ __forceinline__ float col_sum(float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

struct TrainLds {
    Weights W;
    WeightsT T;
    uint16_t x[kBS * kIn], xt[kIn * kLdS];
    uint16_t a1[kBS * kLdH], a1t[kH * kLdS];
    uint16_t a2[kBS * kLdH], a2t[kH * kLdS];
    uint16_t gy[kBS * kOutPad], gyt[kOutPad * kLdS];
    uint16_t gz2[kBS * kLdH], gz2t[kH * kLdS];
    uint16_t gz1t[kH * kLdS];
    float target[kBS * 4];
    float red[4][kH + kH + kOutPad + 1];  // per-wave bias-gradient and loss sums
};

struct TrainArgs {
    Tab t;
    Geo g;
    const uint32_t *slot;
    const uint32_t *train_idx;
    const uint32_t *counts;
    uint64_t seed;
    float gscale;  // 2 / (3 * batch)
};

// one workgroup per compute unit (the LDS it needs): registers are not scarce, so
// the weights' loads can all be issued before the features are computed
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void train_kernel(TrainArgs A, const uint16_t *__restrict__ wb,
                                                          const float *__restrict__ w, float *__restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem[];
    TrainLds &L = *reinterpret_cast<TrainLds *>(smem);
    const uint32_t n_el = A.counts[0];
    float *out = partial + (size_t)blockIdx.x * (kNParam + 1);
    if (n_el == 0) {
        for (int i = threadIdx.x; i < kNParam + 1; i += kThreads) out[i] = 0.0f;
        return;
    }
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4, wave = threadIdx.x >> 6;
    const int r0 = wave * 16;  // this wave's rows of the block tile

    // features and target of sample r0 + lr (4 lanes per sample); the
    // weights' loads go out with the sample's first load and are staged in
    // LDS while the vertex's loads are in flight
    WeightLoads wl;
    {
        const uint32_t j = blockIdx.x * kBS + r0 + lr;
        Pcg32 rng(A.seed, j);
        const uint32_t u = rng.next();
        const uint32_t pick = (uint32_t)(((uint64_t)u * (uint64_t)n_el) >> 32);
        const uint32_t v = A.train_idx[pick];
        wl.issue(wb, w);
        __builtin_amdgcn_sched_barrier(0);  // the weights' loads go out here, not where they are used
        int32_t q[3];
        int lp;
        float x[3], n[3];
        vertex_inputs(A.g, v, q, lp, x, n);
        // the target's cell is requested, and the weights staged, before the
        // features are computed
        pf_cell c;
        if (lg == 0) c = A.t.cell_at(A.slot[v]);
        wl.stage<false>(L.W, &L.T);
        vertex_slots(lg, q, lp, x, n, A.g.cam, [&](int m, uint16_t val) {
            const int f = input_of_lane_value(lg, m);
            L.x[(r0 + lr) * kIn + f] = val;
            L.xt[f * kLdS + r0 + lr] = val;
        });
        if (lg == 0) {
            L.target[(r0 + lr) * 4 + 0] = A.t.average(c, 0);
            L.target[(r0 + lr) * 4 + 1] = A.t.average(c, 1);
            L.target[(r0 + lr) * 4 + 2] = A.t.average(c, 2);
        }
    }
    __syncthreads();

    // forward (this wave's 16 rows)
    v4f z1[4], z2[4];
    const v4f y = forward_tile(L.W, L.x, L.a1, L.a2, kLdH, L.a1t, L.a2t, kLdS, r0, z1, z2);

    // output gradient: gy = 2 (y - t) / (3 B) for the 3 live outputs
    float loss = 0.0f, gyv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = r0 + 4 * lg + i;
        float d = 0.0f;
        if (lr < kOut) d = y[i] - L.target[row * 4 + lr];
        loss += d * d;
        gyv[i] = A.gscale * d;
        L.gy[row * kOutPad + lr] = (uint16_t)bf16x2(gyv[i], 0.0f);
    }
    st4(L.gyt + lr * kLdS + r0 + 4 * lg, gyv[0], gyv[1], gyv[2], gyv[3]);
    {
        const float s3 = col_sum((gyv[0] + gyv[1]) + (gyv[2] + gyv[3]));
        const float sl = col_sum(loss);
        if (lg == 0) L.red[wave][2 * kH + lr] = s3;
        float tot = sl;
        tot += __shfl_xor(tot, 1);
        tot += __shfl_xor(tot, 2);
        tot += __shfl_xor(tot, 4);
        tot += __shfl_xor(tot, 8);
        if (lane == 0) L.red[wave][2 * kH + kOutPad] = tot;
    }
    lds_wait();
    __builtin_amdgcn_wave_barrier();

    // da2 = gy W3, gz2 = da2 * [z2 > 0]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        v4f d = {0, 0, 0, 0};
        d = mfma(ld4(L.gy + (r0 + lr) * kOutPad + 4 * lg), ld4(L.T.w3t + (nt * 16 + lr) * kOutPad + 4 * lg), d);
        const int n = nt * 16 + lr;
        float g[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            g[i] = z2[nt][i] > 0.0f ? d[i] : 0.0f;
            L.gz2[(r0 + 4 * lg + i) * kLdH + n] = (uint16_t)bf16x2(g[i], 0.0f);
        }
        st4(L.gz2t + n * kLdS + r0 + 4 * lg, g[0], g[1], g[2], g[3]);
        const float s = col_sum((g[0] + g[1]) + (g[2] + g[3]));
        if (lg == 0) L.red[wave][kH + n] = s;
    }
    lds_wait();
    __builtin_amdgcn_wave_barrier();

    // da1 = gz2 W2, gz1 = da1 * [z1 > 0]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        v4f d = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < kH / 16; ++kk)
            d = mfma(ld4(L.gz2 + (r0 + lr) * kLdH + kk * 16 + 4 * lg),
                     ld4(L.T.w2t + (nt * 16 + lr) * kLdH + kk * 16 + 4 * lg), d);
        const int n = nt * 16 + lr;
        float g[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) g[i] = z1[nt][i] > 0.0f ? d[i] : 0.0f;
        st4(L.gz1t + n * kLdS + r0 + 4 * lg, g[0], g[1], g[2], g[3]);
        const float s = col_sum((g[0] + g[1]) + (g[2] + g[3]));
        if (lg == 0) L.red[wave][n] = s;
    }
    __syncthreads();

    // weight gradients over the block's 64 samples; wave w owns tiles w, w+4, ...
    // (the partials are stored non-temporally: read once, by the reduction)
    // dW1 [64 x 80]: 20 tiles
    for (int tile = wave; tile < 20; tile += 4) {
        const int mt = tile / 5, nt = tile % 5;
        v4f acc = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < kBS / 16; ++kk)
            acc = mfma(ld4(L.gz1t + (mt * 16 + lr) * kLdS + kk * 16 + 4 * lg),
                       ld4(L.xt + (nt * 16 + lr) * kLdS + kk * 16 + 4 * lg), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) __builtin_nontemporal_store(acc[i], &out[kOffW1 + (mt * 16 + 4 * lg + i) * kIn + nt * 16 + lr]);
    }
    // dW2 [64 x 64]: 16 tiles
    for (int tile = wave; tile < 16; tile += 4) {
        const int mt = tile / 4, nt = tile % 4;
        v4f acc = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < kBS / 16; ++kk)
            acc = mfma(ld4(L.gz2t + (mt * 16 + lr) * kLdS + kk * 16 + 4 * lg),
                       ld4(L.a1t + (nt * 16 + lr) * kLdS + kk * 16 + 4 * lg), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) __builtin_nontemporal_store(acc[i], &out[kOffW2 + (mt * 16 + 4 * lg + i) * kH + nt * 16 + lr]);
    }
    // dW3 [16 x 64]: 4 tiles, one per wave
    {
        const int nt = wave;
        v4f acc = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < kBS / 16; ++kk)
            acc = mfma(ld4(L.gyt + lr * kLdS + kk * 16 + 4 * lg), ld4(L.a2t + (nt * 16 + lr) * kLdS + kk * 16 + 4 * lg),
                       acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) __builtin_nontemporal_store(acc[i], &out[kOffW3 + (4 * lg + i) * kH + nt * 16 + lr]);
    }
    // bias gradients and loss: the 4 waves' sums in wave order
    for (int i = threadIdx.x; i < kH + kH + kOutPad + 1; i += kThreads) {
        const float s = ((L.red[0][i] + L.red[1][i]) + L.red[2][i]) + L.red[3][i];
        int dst;
        if (i < kH) dst = kOffB1 + i;
        else if (i < 2 * kH) dst = kOffB2 + (i - kH);
        else if (i < 2 * kH + kOutPad) dst = kOffB3 + (i - 2 * kH);
        else dst = kNParam;
        __builtin_nontemporal_store(s, &out[dst]);
    }
}

// Sum of the per-workgroup partials, then Adam.  A workgroup of 1024 lanes
// takes 64 parameters; its 16 groups of 64 lanes each sum a contiguous
// sixteenth of the partials (all of a lane's loads in flight together), and
// the 16 group sums are added in a fixed order, so the result is
// deterministic.
constexpr int kRedParams = 64, kRedGroups = 16, kRedThreads = kRedParams * kRedGroups;
__global__ __launch_bounds__(kRedThreads) void reduce_adam_kernel(float *__restrict__ w, uint16_t *__restrict__ wb,
                                                                  float *__restrict__ m, float *__restrict__ v,
                                                                  const float *__restrict__ partial, uint32_t nblocks,
                                                                  const uint32_t *__restrict__ counts, float lr,
                                                                  float c1, float c2, float *__restrict__ loss,
                                                                  float loss_scale) {
    __shared__ float part[kRedGroups][kRedParams];
    if (counts[0] == 0) return;
    const int pl = threadIdx.x % kRedParams, grp = threadIdx.x / kRedParams;
    const int p = blockIdx.x * kRedParams + pl;
    const uint32_t per = (nblocks + kRedGroups - 1) / kRedGroups;
    const uint32_t b0 = grp * per, b1 = min(nblocks, b0 + per);
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (p <= kNParam) {
        for (uint32_t bb = b0; bb < b1; bb += 16) {
            float t[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) t[u] = bb + u < b1 ? partial[(size_t)(bb + u) * (kNParam + 1) + p] : 0.0f;
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u & 7] += t[u];
        }
    }
    part[grp][pl] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    if (grp != 0 || p > kNParam) return;
    float g = 0.0f;
#pragma unroll
    for (int k = 0; k < kRedGroups; ++k) g += part[k][pl];
    if (p == kNParam) {
        loss[0] = g * loss_scale;
        return;
    }
    // 1 - beta as constants of their own: 1.0f - 0.999f is 0.99998713e-3,
    // 1.3e-5 away from Adam's 1 - beta2 = 1e-3
    const float be1 = 0.9f, be2 = 0.999f, omb1 = 0.1f, omb2 = 0.001f, eps = 1e-8f;
    const float mn = be1 * m[p] + omb1 * g;
    const float vn = be2 * v[p] + omb2 * (g * g);
    m[p] = mn;
    v[p] = vn;
    const float mh = mn * c1, vh = vn * c2;
    const float wn = w[p] - lr * mh / (sqrtf(vh) + eps);
    w[p] = wn;
    wb[p] = bf16(wn);
}

// Inference keeps a tile's activations in registers.  Each layer is
// computed transposed, z^T = W a^T, with the weights as the first operand of
// the 16 x 16 x 16 products and the vertices along the columns of the
// second: a lane's result, 4 hidden units of one vertex, is then exactly its
// part of the next layer's second operand, so nothing goes through LDS but
// the weights.
struct InferLds {
    Weights W;
};

__device__ __forceinline__ v4s pack4(float a, float b, float c, float d) {
    const uint2 v = {bf16x2(a, b), bf16x2(c, d)};
    return __builtin_bit_cast(v4s, v);
}

// One wave's 16 vertices: xf[kk] holds this lane's slots 16 kk + 4 lg + i
// of vertex lr.  Returns this lane's 4 outputs 4 lg + i of vertex lr
// (outputs 0..2 live in lane group 0).
__device__ __forceinline__ v4f forward_regs(const Weights &W, const v4s xf[5]) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
    v4s a1[4], a2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        v4f z = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < kIn / 16; ++kk) z = mfma(ld4(W.w1 + (mt * 16 + lr) * kLdIn + kk * 16 + 4 * lg), xf[kk], z);
        const float4 bb = *reinterpret_cast<const float4 *>(W.b1 + mt * 16 + 4 * lg);
        a1[mt] = pack4(fmaxf(z[0] + bb.x, 0.0f), fmaxf(z[1] + bb.y, 0.0f), fmaxf(z[2] + bb.z, 0.0f),
                       fmaxf(z[3] + bb.w, 0.0f));
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        v4f z = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < kH / 16; ++kk) z = mfma(ld4(W.w2 + (mt * 16 + lr) * kLdH + kk * 16 + 4 * lg), a1[kk], z);
        const float4 bb = *reinterpret_cast<const float4 *>(W.b2 + mt * 16 + 4 * lg);
        a2[mt] = pack4(fmaxf(z[0] + bb.x, 0.0f), fmaxf(z[1] + bb.y, 0.0f), fmaxf(z[2] + bb.z, 0.0f),
                       fmaxf(z[3] + bb.w, 0.0f));
    }
    v4f y = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < kH / 16; ++kk) y = mfma(ld4(W.w3 + lr * kLdH + kk * 16 + 4 * lg), a2[kk], y);
    const float4 bb = *reinterpret_cast<const float4 *>(W.b3 + 4 * lg);
    y[0] += bb.x;
    y[1] += bb.y;
    y[2] += bb.z;
    y[3] += bb.w;
    return y;
}

// One workgroup of 16 waves per compute unit: the weights are staged once
// per CU (with four workgroups of 4 waves, the same 20 KB were requested
// four times as often and the staging took up to 24 us behind the L2).
constexpr int kInferThreads = 1024, kInferWaves = kInferThreads / 64;
__global__ __launch_bounds__(kInferThreads) void infer_kernel(Geo g, const uint16_t *__restrict__ wb,
                                                          const float *__restrict__ w, const uint32_t *idx,
                                                          const uint32_t *counts, float *r, float *gc, float *b) {
    extern __shared__ __align__(16) unsigned char smem[];
    InferLds &L = *reinterpret_cast<InferLds *>(smem);
    const uint32_t n = counts[1];
    if (n == 0) return;
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4, wave = threadIdx.x >> 6;
    {
        WeightLoadsT<kInferThreads> wl;
        wl.issue(wb, w);
        wl.stage<true>(L.W, nullptr);
    }
    __syncthreads();

    // Tiles of 16 listed vertices, strided over the waves.  The loads are
    // software-pipelined: a tile's vertex inputs are requested one tile
    // ahead and its list entries two tiles ahead, so that the two dependent
    // random loads before a tile's features overlap the tiles before it.
    const uint32_t ntiles = (n + 15) / 16;
    const uint32_t stride = gridDim.x * kInferWaves;
    constexpr uint32_t kNone = 0xffffffffu;
    auto entry = [&](uint32_t t) -> uint32_t {  // this lane's vertex in tile t (kNone: none)
        const uint32_t e = t * 16 + lr;
        return t < ntiles && e < n ? idx[e] : kNone;
    };
    struct In {
        uint64_t key;
        float x[3], nv[3];
    };
    auto inputs = [&](uint32_t vtx) {
        In in;
        const uint32_t v = vtx != kNone ? vtx : 0u;  // a lane of no vertex reads vertex 0, unused
        in.key = g.key[v];
        in.x[0] = g.px[v];
        in.x[1] = g.py[v];
        in.x[2] = g.pz[v];
        in.nv[0] = g.nx[v];
        in.nv[1] = g.ny[v];
        in.nv[2] = g.nz[v];
        return in;
    };
    uint32_t tile = blockIdx.x * kInferWaves + wave;
    uint32_t vtx = entry(tile);
    In cur = inputs(vtx);
    uint32_t vtx_next = entry(tile + stride);
    for (; tile < ntiles; tile += stride) {
        const In nxt = inputs(vtx_next);
        const uint32_t vtx_after = entry(tile + 2 * stride);
        int32_t q[3];
        q[0] = (int32_t)((cur.key >> 0) & 0x1ffffu) - 65536;
        q[1] = (int32_t)((cur.key >> 17) & 0x1ffffu) - 65536;
        q[2] = (int32_t)((cur.key >> 34) & 0x1ffffu) - 65536;
        const int lp = (int)((cur.key >> 51) & 31u) - 16;
        v4s xf[5];
        vertex_slots(lg, q, lp, cur.x, cur.nv, g.cam, [&](int m, uint16_t val) { xf[m >> 2][m & 3] = (short)val; });
        // the weights are read from LDS in every tile: an offset the compiler
        // cannot see through keeps it from holding all of them in registers
        // (which would leave two waves a SIMD)
        uint32_t wofs = 0;
        asm volatile("" : "+v"(wofs));
        const v4f y = forward_regs(*reinterpret_cast<const Weights *>(smem + wofs), xf);
        if (lg == 0 && vtx != kNone && isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2])) {
            r[vtx] = y[0] > 0.0f ? y[0] : 0.0f;
            gc[vtx] = y[1] > 0.0f ? y[1] : 0.0f;
            b[vtx] = y[2] > 0.0f ? y[2] : 0.0f;
        }
        cur = nxt;
        vtx = vtx_next;
        vtx_next = vtx_after;
    }
}

// Features of listed vertices, one thread per (vertex, feature).
__global__ __launch_bounds__(kThreads) void features_kernel(Geo g, const uint32_t *idx, uint32_t n,
                                                             uint16_t *out) {
    const uint64_t t = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= (uint64_t)n * kIn) return;
    const uint32_t e = (uint32_t)(t / kIn);
    const int f = (int)(t % kIn);
    int32_t q[3];
    int lp;
    float x[3], nv[3];
    vertex_inputs(g, idx[e], q, lp, x, nv);
    out[t] = feature(f, q, lp, x, nv, g.cam);
}

__global__ void init_kernel(const float *__restrict__ w, uint16_t *__restrict__ wb, float *__restrict__ m,
                            float *__restrict__ v, float *__restrict__ loss) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p < kNParam) {
        wb[p] = bf16(w[p]);
        m[p] = 0.0f;
        v[p] = 0.0f;
    }
    if (p == 0) loss[0] = 0.0f;
}

// ----------------------------------------------------------- selection
// Two passes over blocks of 4096 vertices, 16 consecutive vertices a thread.
// The first reads the flags and counts (one 16-byte load of flags, four of
// counts where both arrays are 16-byte aligned), counts each block's listed
// vertices and keeps each thread's two 16-bit masks in one word (1 bit per
// vertex and list instead of the 5 bytes read).  The second reads the masks,
// sums the counts of the blocks before its own (a few KB from L2, so there
// is no separate scan), ranks its threads, and writes its part of each list
// as one contiguous run staged in LDS, in vertex order.
constexpr int kSelPerThread = 16;
constexpr int kSelPerBlock = kThreads * kSelPerThread;  // 4096

// Bit v of tr / sp: vertex base + v is listed for training / as sparse.
__device__ __forceinline__ void sel_masks(uint32_t base, uint32_t n, const uint8_t *flags, const uint32_t *count,
                                          uint32_t lo, uint32_t hi, bool vec, uint32_t &tr, uint32_t &sp) {
    tr = sp = 0;
    if (vec && base + kSelPerThread <= n) {
        const uint4 f4 = *reinterpret_cast<const uint4 *>(flags + base);
        const uint32_t fw[4] = {f4.x, f4.y, f4.z, f4.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 c4 = *reinterpret_cast<const uint4 *>(count + base + 4 * q);
            const uint32_t cw[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool ok = ((fw[q] >> (8 * k)) & 0xffu) == 0;
                tr |= (uint32_t)(ok && cw[k] >= hi) << (4 * q + k);
                sp |= (uint32_t)(ok && cw[k] < lo) << (4 * q + k);
            }
        }
    } else {
        for (int v = 0; v < kSelPerThread; ++v) {
            const uint32_t i = base + v;
            if (i < n && flags[i] == 0) {
                const uint32_t c = count[i];
                tr |= (uint32_t)(c >= hi) << v;
                sp |= (uint32_t)(c < lo) << v;
            }
        }
    }
}

// Block-wide exclusive prefix (in thread order) of a and b, and the totals.
__device__ __forceinline__ void block_scan2(uint32_t a, uint32_t b, uint32_t &pa, uint32_t &pb, uint32_t &ta,
                                            uint32_t &tb) {
    __shared__ uint32_t s_wave[2][kThreads / 64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t ia = a, ib = b;
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t ua = __shfl_up(ia, off), ub = __shfl_up(ib, off);
        if (lane >= off) {
            ia += ua;
            ib += ub;
        }
    }
    if (lane == 63) {
        s_wave[0][wave] = ia;
        s_wave[1][wave] = ib;
    }
    __syncthreads();
    uint32_t wa = 0, wb = 0;
    ta = tb = 0;
    for (uint32_t k = 0; k < kThreads / 64; ++k) {
        if (k < wave) {
            wa += s_wave[0][k];
            wb += s_wave[1][k];
        }
        ta += s_wave[0][k];
        tb += s_wave[1][k];
    }
    pa = wa + ia - a;
    pb = wb + ib - b;
    __syncthreads();  // s_wave is reused by the next call
}

// bcnt: [0, nblocks) training counts, [nblocks, 2 nblocks) sparse counts,
// then a word per thread: training mask (low 16 bits), sparse mask (high)
__global__ __launch_bounds__(kThreads) void select_count_kernel(const uint8_t *flags, const uint32_t *count,
                                                                uint32_t n, uint32_t lo, uint32_t hi, bool vec,
                                                                uint32_t *bcnt, uint32_t nblocks) {
    uint32_t tr, sp;
    sel_masks(blockIdx.x * kSelPerBlock + threadIdx.x * kSelPerThread, n, flags, count, lo, hi, vec, tr, sp);
    bcnt[2 * nblocks + blockIdx.x * kThreads + threadIdx.x] = tr | sp << 16;
    uint32_t pa, pb, ta, tb;
    block_scan2(__popc(tr), __popc(sp), pa, pb, ta, tb);
    if (threadIdx.x == 0) {
        bcnt[blockIdx.x] = ta;
        bcnt[nblocks + blockIdx.x] = tb;
    }
}

__global__ __launch_bounds__(kThreads) void select_scatter_kernel(const uint32_t *bcnt, uint32_t nblocks,
                                                                  uint32_t *tr_idx, uint32_t *sp_idx,
                                                                  uint32_t *counts) {
    const uint32_t base = blockIdx.x * kSelPerBlock + threadIdx.x * kSelPerThread;
    uint32_t tr = 0, sp = 0;
    if (nblocks) {
        const uint32_t m = bcnt[2 * nblocks + blockIdx.x * kThreads + threadIdx.x];
        tr = m & 0xffffu;
        sp = m >> 16;
    }
    // this block's offsets: the counts of the blocks before it
    uint32_t before_t = 0, before_s = 0;
    for (uint32_t k = threadIdx.x; k < blockIdx.x; k += kThreads) {
        before_t += bcnt[k];
        before_s += bcnt[nblocks + k];
    }
    uint32_t dummy_a, dummy_b, off_t, off_s;
    block_scan2(before_t, before_s, dummy_a, dummy_b, off_t, off_s);
    uint32_t pt, ps, tt, ts;
    block_scan2(__popc(tr), __popc(sp), pt, ps, tt, ts);
    if (blockIdx.x + 1 == gridDim.x && threadIdx.x == 0) {  // the last block knows the totals
        counts[0] = off_t + tt;
        counts[1] = off_s + ts;
    }
    // the block's entries go to LDS in order, then out as two contiguous runs
    __shared__ uint32_t s_tr[kSelPerBlock], s_sp[kSelPerBlock];
    uint32_t ot = pt, os = ps;
    for (int v = 0; v < kSelPerThread; ++v) {
        if ((tr >> v) & 1u) s_tr[ot++] = base + v;
        if ((sp >> v) & 1u) s_sp[os++] = base + v;
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < tt; k += kThreads) tr_idx[off_t + k] = s_tr[k];
    for (uint32_t k = threadIdx.x; k < ts; k += kThreads) sp_idx[off_s + k] = s_sp[k];
}

}  // namespace mlp

// ----------------------------------------------------------- launchers
hipError_t launch_mlp_init(const MlpArgs &a, hipStream_t st) {
    mlp::init_kernel<<<(mlp::kNParam + mlp::kThreads - 1) / mlp::kThreads, mlp::kThreads, 0, st>>>(a.w, a.wb, a.m,
                                                                                                  a.v, a.loss);
    return hipGetLastError();
}

hipError_t launch_mlp_select(const uint8_t *flags, const uint32_t *count, uint32_t n, uint32_t lo, uint32_t hi,
                             uint32_t *tr_idx, uint32_t *sp_idx, uint32_t *counts, uint32_t *ws, hipStream_t st) {
    const uint32_t nblocks = (n + mlp::kSelPerBlock - 1) / mlp::kSelPerBlock;
    // 16-byte loads where both arrays allow them (the blocks start on
    // multiples of 4096 vertices)
    const bool vec = reinterpret_cast<uintptr_t>(flags) % 16 == 0 && reinterpret_cast<uintptr_t>(count) % 16 == 0;
    if (nblocks)
        mlp::select_count_kernel<<<nblocks, mlp::kThreads, 0, st>>>(flags, count, n, lo, hi, vec, ws, nblocks);
    // n == 0: one block writes zero counts
    mlp::select_scatter_kernel<<<nblocks ? nblocks : 1, mlp::kThreads, 0, st>>>(ws, nblocks, tr_idx, sp_idx,
                                                                                counts);
    return hipGetLastError();
}

uint32_t mlp_select_blocks(uint32_t n) { return (n + mlp::kSelPerBlock - 1) / mlp::kSelPerBlock; }

hipError_t launch_mlp_train(const MlpArgs &a, const Tab &t, const GeoArgs &g, const uint32_t *slot,
                            const uint32_t *train_idx, const uint32_t *counts, uint32_t batch, uint64_t seed,
                            uint32_t step, float lr, hipStream_t st) {
    mlp::TrainArgs A;
    A.t = t;
    A.g.key = g.key;
    A.g.px = g.px;
    A.g.py = g.py;
    A.g.pz = g.pz;
    A.g.nx = g.nx;
    A.g.ny = g.ny;
    A.g.nz = g.nz;
    for (int c = 0; c < 3; ++c) A.g.cam[c] = g.cam[c];
    A.slot = slot;
    A.train_idx = train_idx;
    A.counts = counts;
    A.seed = seed;
    A.gscale = (float)(2.0 / (3.0 * (double)batch));
    const uint32_t nblocks = batch / mlp::kBS;
    const size_t lds = sizeof(mlp::TrainLds);
    static bool lds_set = false;  // the attribute is per function: set it once
    if (!lds_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(mlp::train_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = true;
    }
    mlp::train_kernel<<<nblocks, mlp::kThreads, lds, st>>>(A, a.wb, a.w, a.partial);
    const double c1 = 1.0 / (1.0 - pow(0.9, (double)step));
    const double c2 = 1.0 / (1.0 - pow(0.999, (double)step));
    mlp::reduce_adam_kernel<<<(mlp::kNParam + 1 + mlp::kRedParams - 1) / mlp::kRedParams, mlp::kRedThreads, 0, st>>>(
        a.w, a.wb, a.m, a.v, a.partial, nblocks, counts, lr, (float)c1, (float)c2, a.loss,
        (float)(1.0 / (3.0 * (double)batch)));
    return hipGetLastError();
}

hipError_t launch_mlp_features(const GeoArgs &g, const uint32_t *idx, uint32_t n, uint16_t *out, hipStream_t st) {
    mlp::Geo G;
    G.key = g.key;
    G.px = g.px;
    G.py = g.py;
    G.pz = g.pz;
    G.nx = g.nx;
    G.ny = g.ny;
    G.nz = g.nz;
    for (int c = 0; c < 3; ++c) G.cam[c] = g.cam[c];
    const uint64_t total = (uint64_t)n * mlp::kIn;
    mlp::features_kernel<<<(uint32_t)((total + mlp::kThreads - 1) / mlp::kThreads), mlp::kThreads, 0, st>>>(G, idx, n,
                                                                                                           out);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const MlpArgs &a, const GeoArgs &g, const uint32_t *idx, const uint32_t *counts,
                            uint32_t n_max, float *r, float *gc, float *b, hipStream_t st) {
    mlp::Geo G;
    G.key = g.key;
    G.px = g.px;
    G.py = g.py;
    G.pz = g.pz;
    G.nx = g.nx;
    G.ny = g.ny;
    G.nz = g.nz;
    for (int c = 0; c < 3; ++c) G.cam[c] = g.cam[c];
    const size_t lds = sizeof(mlp::InferLds);
    static bool lds_set = false;  // the attribute is per function: set it once
    if (!lds_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(mlp::infer_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = true;
    }
    // no more workgroups than are resident at once: the waves stride over
    // the tiles, and a second round of workgroups would start only when the
    // first has finished (per device, asked once)
    static uint32_t resident[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (resident[dev] == 0) {
        int per_cu = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(mlp::infer_kernel),
                                                         mlp::kInferThreads, lds);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        resident[dev] = (uint32_t)(per_cu > 0 ? per_cu : 1) * (uint32_t)(cus > 0 ? cus : 1);
    }
    const uint32_t tiles = (n_max + 15) / 16;
    uint32_t blocks = (tiles + mlp::kInferWaves - 1) / mlp::kInferWaves;
    if (blocks > resident[dev]) blocks = resident[dev];
    if (blocks == 0) blocks = 1;
    mlp::infer_kernel<<<blocks, mlp::kInferThreads, lds, st>>>(G, a.wb, a.w, idx, counts, r, gc, b);
    return hipGetLastError();
}

}  // namespace pfk
