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
constexpr int kLdH = kH + 8;   // rows of 64 hidden units (weights W2, W3, W2^T; activations)
constexpr int kLdS = kBS + 8;  // rows of 64 samples (transposed operands)
constexpr int kThreads = 256;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// float -> bfloat16, round to nearest even, NaN kept quiet
__device__ __forceinline__ uint16_t bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ v4s ld4(const uint16_t *p) { return *reinterpret_cast<const v4s *>(p); }

__device__ __forceinline__ void st4(uint16_t *p, float a, float b, float c, float d) {
    v4s v;
    v.x = (short)bf16(a);
    v.y = (short)bf16(b);
    v.z = (short)bf16(c);
    v.w = (short)bf16(d);
    *reinterpret_cast<v4s *>(p) = v;
}

// FP64 -> FP32 -> BF16, zeros as +0 (sinpi and cospi may return -0)
__device__ __forceinline__ uint16_t to_feature(double v) {
    v = v + 0.0;
    return bf16((float)v);
}

// Positional-encoding pair j of coordinate c: sin and cos of pi t with the
// exact phase t = (q + 1/2) 2^(lp - 10 + j) = (2q + 1) 2^e, e = lp - 11 + j.
// For e >= 0 the phase is an integer (even for e >= 1) and the values are
// 0 and +-1 exactly; otherwise one FP64 sincospi gives both.
__device__ __forceinline__ void pe_pair(int32_t qc, int lp, int j, uint16_t &sv, uint16_t &cv) {
    const int e = lp - 11 + j;
    double sn = 0.0, cs = 1.0;
    if (e == 0) {
        cs = -1.0;  // odd integer
    } else if (e < 0) {
        const double t = ldexp((double)qc + 0.5, lp - 10 + j);  // exact
        sincospi(t, &sn, &cs);
    }
    sv = to_feature(sn);
    cv = to_feature(cs);
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

// The 80 features of one vertex, computed by the 4 lanes lg = 0..3 of its
// group: lane lg takes the positional pairs lg, lg + 4, ... (9 of the 36)
// and features 72 + lg and 76 + lg; put(f, value) stores feature f.
template <typename Put>
__device__ __forceinline__ void vertex_features(int lg, const int32_t q[3], int lp, const float x[3],
                                                const float n[3], const float cam[3], Put put) {
    for (int pi = lg; pi < 36; pi += 4) {
        const int j = pi / 3, c = pi % 3;
        uint16_t sv, cv;
        pe_pair(q[c], lp, j, sv, cv);
        put(6 * j + c, sv);
        put(6 * j + 3 + c, cv);
    }
    put(72 + lg, feature(72 + lg, q, lp, x, n, cam));
    put(76 + lg, feature(76 + lg, q, lp, x, n, cam));
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
    uint16_t w1[kH * kIn];
    uint16_t w2[kH * kLdH];
    uint16_t w3[kOutPad * kLdH];
    float b1[kH], b2[kH], b3[kOutPad];
};

struct WeightsT {
    uint16_t w2t[kH * kLdH];
    uint16_t w3t[kH * kOutPad];
};

__device__ void load_weights(Weights &W, WeightsT *T, const uint16_t *wb, const float *w) {
    for (int i = threadIdx.x; i < kH * kIn; i += kThreads) W.w1[i] = wb[kOffW1 + i];
    for (int i = threadIdx.x; i < kH * kH; i += kThreads) {
        const uint16_t val = wb[kOffW2 + i];
        W.w2[(i / kH) * kLdH + i % kH] = val;
        if (T) T->w2t[(i % kH) * kLdH + i / kH] = val;
    }
    for (int i = threadIdx.x; i < kOutPad * kH; i += kThreads) {
        const uint16_t val = wb[kOffW3 + i];
        W.w3[(i / kH) * kLdH + i % kH] = val;
        if (T) T->w3t[(i % kH) * kOutPad + i / kH] = val;
    }
    for (int i = threadIdx.x; i < kH; i += kThreads) {
        W.b1[i] = w[kOffB1 + i];
        W.b2[i] = w[kOffB2 + i];
    }
    for (int i = threadIdx.x; i < kOutPad; i += kThreads) W.b3[i] = w[kOffB3 + i];
}

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
        for (int nt = 0; nt < 4; ++nt) z1[nt] = mfma(a, ld4(W.w1 + (nt * 16 + lr) * kIn + kk * 16 + 4 * lg), z1[nt]);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int n = nt * 16 + lr;
        float h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            z1[nt][i] += W.b1[n];
            h[i] = z1[nt][i] > 0.0f ? z1[nt][i] : 0.0f;
            a1[(r0 + 4 * lg + i) * lda + n] = bf16(h[i]);
        }
        if (a1t) st4(a1t + n * ldt + r0 + 4 * lg, h[0], h[1], h[2], h[3]);
    }
    __builtin_amdgcn_s_waitcnt(0);
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
            a2[(r0 + 4 * lg + i) * lda + n] = bf16(h[i]);
        }
        if (a2t) st4(a2t + n * ldt + r0 + 4 * lg, h[0], h[1], h[2], h[3]);
    }
    __builtin_amdgcn_s_waitcnt(0);
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

__global__ __launch_bounds__(kThreads) void train_kernel(TrainArgs A, const uint16_t *__restrict__ wb,
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

    load_weights(L.W, &L.T, wb, w);

    // features and target of sample r0 + lr (4 lanes per sample)
    {
        const uint32_t j = blockIdx.x * kBS + r0 + lr;
        Pcg32 rng(A.seed, j);
        const uint32_t u = rng.next();
        const uint32_t pick = (uint32_t)(((uint64_t)u * (uint64_t)n_el) >> 32);
        const uint32_t v = A.train_idx[pick];
        int32_t q[3];
        int lp;
        float x[3], n[3];
        vertex_inputs(A.g, v, q, lp, x, n);
        vertex_features(lg, q, lp, x, n, A.g.cam, [&](int f, uint16_t val) {
            L.x[(r0 + lr) * kIn + f] = val;
            L.xt[f * kLdS + r0 + lr] = val;
        });
        if (lg == 0) {
            const pf_cell c = A.t.cell_at(A.slot[v]);
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
        L.gy[row * kOutPad + lr] = bf16(gyv[i]);
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
    __builtin_amdgcn_s_waitcnt(0);
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
            L.gz2[(r0 + 4 * lg + i) * kLdH + n] = bf16(g[i]);
        }
        st4(L.gz2t + n * kLdS + r0 + 4 * lg, g[0], g[1], g[2], g[3]);
        const float s = col_sum((g[0] + g[1]) + (g[2] + g[3]));
        if (lg == 0) L.red[wave][kH + n] = s;
    }
    __builtin_amdgcn_s_waitcnt(0);
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
    // dW1 [64 x 80]: 20 tiles
    for (int tile = wave; tile < 20; tile += 4) {
        const int mt = tile / 5, nt = tile % 5;
        v4f acc = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < kBS / 16; ++kk)
            acc = mfma(ld4(L.gz1t + (mt * 16 + lr) * kLdS + kk * 16 + 4 * lg),
                       ld4(L.xt + (nt * 16 + lr) * kLdS + kk * 16 + 4 * lg), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) out[kOffW1 + (mt * 16 + 4 * lg + i) * kIn + nt * 16 + lr] = acc[i];
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
        for (int i = 0; i < 4; ++i) out[kOffW2 + (mt * 16 + 4 * lg + i) * kH + nt * 16 + lr] = acc[i];
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
        for (int i = 0; i < 4; ++i) out[kOffW3 + (4 * lg + i) * kH + nt * 16 + lr] = acc[i];
    }
    // bias gradients and loss: the 4 waves' sums in wave order
    for (int i = threadIdx.x; i < kH + kH + kOutPad + 1; i += kThreads) {
        const float s = ((L.red[0][i] + L.red[1][i]) + L.red[2][i]) + L.red[3][i];
        int dst;
        if (i < kH) dst = kOffB1 + i;
        else if (i < 2 * kH) dst = kOffB2 + (i - kH);
        else if (i < 2 * kH + kOutPad) dst = kOffB3 + (i - 2 * kH);
        else dst = kNParam;
        out[dst] = s;
    }
}

// Sum of the per-workgroup partials, then Adam.  A workgroup takes 64
// parameters; its four groups of 64 lanes each sum a contiguous quarter of
// the partials (independent loads in flight together), and the four
// quarter sums are added in a fixed order, so the result is deterministic.
constexpr int kRedParams = 64;
__global__ __launch_bounds__(kThreads) void reduce_adam_kernel(float *__restrict__ w, uint16_t *__restrict__ wb,
                                                               float *__restrict__ m, float *__restrict__ v,
                                                               const float *__restrict__ partial, uint32_t nblocks,
                                                               const uint32_t *__restrict__ counts, float lr,
                                                               float c1, float c2, float *__restrict__ loss,
                                                               float loss_scale) {
    static_assert(kThreads == 4 * kRedParams, "four groups of 64 lanes");
    __shared__ float quarter[4][kRedParams];
    if (counts[0] == 0) return;
    const int pl = threadIdx.x % kRedParams, grp = threadIdx.x / kRedParams;
    const int p = blockIdx.x * kRedParams + pl;
    const uint32_t per = (nblocks + 3) / 4;
    const uint32_t b0 = grp * per, b1 = min(nblocks, b0 + per);
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (p <= kNParam) {
        uint32_t bb = b0;
        for (; bb + 8 <= b1; bb += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += partial[(size_t)(bb + u) * (kNParam + 1) + p];
        }
        for (; bb < b1; ++bb) acc[0] += partial[(size_t)bb * (kNParam + 1) + p];
    }
    quarter[grp][pl] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    if (grp != 0 || p > kNParam) return;
    const float g = (quarter[0][pl] + quarter[1][pl]) + (quarter[2][pl] + quarter[3][pl]);
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

// Per wave: the tile's features (then, once layer 1 has read them, its
// outputs) and one activation buffer that layer 2 overwrites after reading
// it (all of a wave's reads of a1 complete before its first write), so
// that four workgroups fit a CU.
struct InferLds {
    Weights W;
    uint16_t x[4 * 16 * kIn];
    uint16_t a1[4 * 16 * kH];
};
static_assert(16 * kIn * sizeof(uint16_t) >= 16 * kOutPad * sizeof(float), "outputs fit a wave's feature rows");

__global__ __launch_bounds__(kThreads) void infer_kernel(Geo g, const uint16_t *__restrict__ wb,
                                                          const float *__restrict__ w, const uint32_t *idx,
                                                          const uint32_t *counts, float *r, float *gc, float *b) {
    extern __shared__ __align__(16) unsigned char smem[];
    InferLds &L = *reinterpret_cast<InferLds *>(smem);
    const uint32_t n = counts[1];
    if (n == 0) return;
    load_weights(L.W, nullptr, wb, w);
    __syncthreads();
    const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4, wave = threadIdx.x >> 6;
    uint16_t *x = L.x + wave * 16 * kIn;
    uint16_t *a1 = L.a1 + wave * 16 * kH;
    uint16_t *a2 = a1;
    float *yb = reinterpret_cast<float *>(x);
    const uint32_t ntiles = (n + 15) / 16;
    for (uint32_t tile = blockIdx.x * 4 + wave; tile < ntiles; tile += gridDim.x * 4) {
        const uint32_t e = tile * 16 + lr;
        const bool live = e < n;
        const uint32_t vtx = live ? idx[e] : 0u;
        if (live) {
            int32_t q[3];
            int lp;
            float xv[3], nv[3];
            vertex_inputs(g, vtx, q, lp, xv, nv);
            vertex_features(lg, q, lp, xv, nv, g.cam, [&](int f, uint16_t val) { x[lr * kIn + f] = val; });
        } else {
            for (int f = lg; f < kIn; f += 4) x[lr * kIn + f] = 0;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        v4f z1[4], z2[4];
        const v4f y = forward_tile(L.W, x, a1, a2, kH, nullptr, nullptr, 0, 0, z1, z2);
#pragma unroll
        for (int i = 0; i < 4; ++i) yb[(4 * lg + i) * kOutPad + lr] = y[i];
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        if (lg == 0 && live) {
            const float y0 = yb[lr * kOutPad + 0], y1 = yb[lr * kOutPad + 1], y2 = yb[lr * kOutPad + 2];
            if (isfinite(y0) && isfinite(y1) && isfinite(y2)) {
                r[vtx] = y0 > 0.0f ? y0 : 0.0f;
                gc[vtx] = y1 > 0.0f ? y1 : 0.0f;
                b[vtx] = y2 > 0.0f ? y2 : 0.0f;
            }
        }
        __builtin_amdgcn_wave_barrier();
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
constexpr int kSelPerBlock = 1024;  // 256 threads x 4 vertices

__device__ __forceinline__ void sel_pred(uint32_t i, uint32_t n, const uint8_t *flags, const uint32_t *count,
                                         uint32_t lo, uint32_t hi, bool &tr, bool &sp) {
    tr = sp = false;
    if (i < n && flags[i] == 0) {
        const uint32_t c = count[i];
        tr = c >= hi;
        sp = c < lo;
    }
}

__global__ __launch_bounds__(kThreads) void select_count_kernel(const uint8_t *flags, const uint32_t *count,
                                                                uint32_t n, uint32_t lo, uint32_t hi,
                                                                uint32_t *bcnt, uint32_t nblocks) {
    __shared__ uint32_t s_t[4], s_s[4];
    uint32_t ct = 0, cs = 0;
    for (int k = 0; k < 4; ++k) {
        bool tr, sp;
        sel_pred(blockIdx.x * kSelPerBlock + k * kThreads + threadIdx.x, n, flags, count, lo, hi, tr, sp);
        ct += __popcll(__ballot(tr));
        cs += __popcll(__ballot(sp));
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_t[wave] = ct;
        s_s[wave] = cs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bcnt[blockIdx.x] = s_t[0] + s_t[1] + s_t[2] + s_t[3];
        bcnt[nblocks + blockIdx.x] = s_s[0] + s_s[1] + s_s[2] + s_s[3];
    }
}

// One workgroup: exclusive scan of both per-block count arrays (in place)
// and the totals into counts[0..1].
__global__ __launch_bounds__(1024) void select_scan_kernel(uint32_t *bcnt, uint32_t nblocks, uint32_t *counts) {
    __shared__ uint32_t s_sum[2][1024];
    const uint32_t per = (nblocks + 1023) / 1024;
    for (int list = 0; list < 2; ++list) {
        uint32_t *c = bcnt + list * nblocks;
        const uint32_t b0 = threadIdx.x * per;
        uint32_t local = 0;
        for (uint32_t k = 0; k < per; ++k)
            if (b0 + k < nblocks) local += c[b0 + k];
        s_sum[list][threadIdx.x] = local;
    }
    __syncthreads();
    // exclusive scan of the 1024 partials of each list: inclusive scans
    // within each wavefront (shuffles), then over the 16 wavefront totals
    __shared__ uint32_t s_wave[2][16];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl[2];
    for (int list = 0; list < 2; ++list) {
        uint32_t v = s_sum[list][threadIdx.x];
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t o = __shfl_up(v, off);
            if (lane >= off) v += o;
        }
        incl[list] = v;
        if (lane == 63) s_wave[list][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 2) {  // 16 wavefront totals per list
        uint32_t run = 0;
        for (int k = 0; k < 16; ++k) {
            const uint32_t t = s_wave[threadIdx.x][k];
            s_wave[threadIdx.x][k] = run;
            run += t;
        }
        counts[threadIdx.x] = run;
    }
    __syncthreads();
    for (int list = 0; list < 2; ++list)
        s_sum[list][threadIdx.x] = s_wave[list][wave] + incl[list] - s_sum[list][threadIdx.x];
    __syncthreads();
    for (int list = 0; list < 2; ++list) {
        uint32_t *c = bcnt + list * nblocks;
        const uint32_t b0 = threadIdx.x * per;
        uint32_t run = s_sum[list][threadIdx.x];
        for (uint32_t k = 0; k < per; ++k)
            if (b0 + k < nblocks) {
                const uint32_t t = c[b0 + k];
                c[b0 + k] = run;
                run += t;
            }
    }
}

__global__ __launch_bounds__(kThreads) void select_scatter_kernel(const uint8_t *flags, const uint32_t *count,
                                                                  uint32_t n, uint32_t lo, uint32_t hi,
                                                                  const uint32_t *boff, uint32_t nblocks,
                                                                  uint32_t *tr_idx, uint32_t *sp_idx) {
    __shared__ uint32_t s_t[4], s_s[4];
    uint32_t base_t = boff[blockIdx.x], base_s = boff[nblocks + blockIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = 0; k < 4; ++k) {
        const uint32_t i = blockIdx.x * kSelPerBlock + k * kThreads + threadIdx.x;
        bool tr, sp;
        sel_pred(i, n, flags, count, lo, hi, tr, sp);
        const uint64_t bt = __ballot(tr), bs = __ballot(sp);
        if (lane == 0) {
            s_t[wave] = __popcll(bt);
            s_s[wave] = __popcll(bs);
        }
        __syncthreads();
        uint32_t ot = base_t, os = base_s;
        for (int w2 = 0; w2 < wave; ++w2) {
            ot += s_t[w2];
            os += s_s[w2];
        }
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if (tr) tr_idx[ot + __popcll(bt & below)] = i;
        if (sp) sp_idx[os + __popcll(bs & below)] = i;
        base_t += s_t[0] + s_t[1] + s_t[2] + s_t[3];
        base_s += s_s[0] + s_s[1] + s_s[2] + s_s[3];
        __syncthreads();
    }
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
    if (nblocks) mlp::select_count_kernel<<<nblocks, mlp::kThreads, 0, st>>>(flags, count, n, lo, hi, ws, nblocks);
    mlp::select_scan_kernel<<<1, 1024, 0, st>>>(ws, nblocks, counts);  // n == 0: writes zero counts
    if (nblocks)
        mlp::select_scatter_kernel<<<nblocks, mlp::kThreads, 0, st>>>(flags, count, n, lo, hi, ws, nblocks, tr_idx,
                                                                      sp_idx);
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
    mlp::reduce_adam_kernel<<<(mlp::kNParam + 1 + mlp::kRedParams - 1) / mlp::kRedParams, mlp::kThreads, 0, st>>>(
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
    const uint32_t tiles = (n_max + 15) / 16;
    uint32_t blocks = (tiles + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) blocks = 1;
    const size_t lds = sizeof(mlp::InferLds);
    static bool lds_set = false;  // the attribute is per function: set it once
    if (!lds_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(mlp::infer_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        lds_set = true;
    }
    mlp::infer_kernel<<<blocks, mlp::kThreads, lds, st>>>(G, a.wb, a.w, idx, counts, r, gc, b);
    return hipGetLastError();
}

}  // namespace pfk
