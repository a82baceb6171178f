// Key construction (Algorithm 1) for gfx950: one vertex per lane, coalesced
// structure-of-arrays streams in, 8-byte keys and 1-byte flags out.
#include "pf_device.h"
#include "pf_kernels.h"

namespace pfk {

__global__ __launch_bounds__(kBlock) void build_keys_kernel(
    const float *__restrict__ px, const float *__restrict__ py, const float *__restrict__ pz,
    const float *__restrict__ nx, const float *__restrict__ ny, const float *__restrict__ nz,
    const uint8_t *__restrict__ valid, uint32_t n, KeyArgs a, uint64_t *__restrict__ key_out,
    uint32_t *__restrict__ fp_out, uint32_t *__restrict__ home_out, uint8_t *__restrict__ flags_out) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;

    const float x[3] = {px[i], py[i], pz[i]};
    const float nr[3] = {nx[i], ny[i], nz[i]};
    const bool ok_in = (valid == nullptr || valid[i] != 0) && isfinite(x[0]) && isfinite(x[1]) &&
                       isfinite(x[2]) && isfinite(nr[0]) && isfinite(nr[1]) && isfinite(nr[2]);
    uint64_t key = 0;
    uint32_t fp = 0, home = 0;
    uint8_t flags = PF_V_INVALID;
    if (ok_in) {
        // l <- level_of_detail(|p_cam - x|)
        const int l = level_of_detail(a.cam[0], a.cam[1], a.cam[2], x[0], x[1], x[2]);
        // jitter(n): cube sample projected onto the tangent plane
        Pcg32 g(a.seed, a.idx_base + i);
        float r[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = ldexpf((float)(g.next() >> 8), -24) - 0.5f;
        const float t0 = r[0] * nr[0];
        const float t1 = r[1] * nr[1];
        const float t2 = r[2] * nr[2];
        const float t = (t0 + t1) + t2;
        // x' <- x + jitter(n) * s * 2^l
        const float h = ldexpf(a.s, l);
        float xp[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float tn = t * nr[c];
            const float j = r[c] - tn;
            const float jh = j * h;
            xp[c] = x[c] + jh;
        }
        // l' <- level_of_detail(|p_cam - x'|); x~ <- floor(x' / (s * 2^l'))
        const int lp = level_of_detail(a.cam[0], a.cam[1], a.cam[2], xp[0], xp[1], xp[2]);
        const float hp = ldexpf(a.s, lp);
        bool inrange = true;
        int32_t q[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float f = floorf(xp[c] / hp);
            inrange = inrange && (f >= -kCellIndexLimit) && (f < kCellIndexLimit);
            q[c] = inrange ? (int32_t)f : 0;
        }
        if (inrange) {
            const uint32_t code = normal_class(nr[0]) | (normal_class(nr[1]) << 2) | (normal_class(nr[2]) << 4);
            key = (uint64_t)(uint32_t)(q[0] + 65536) | ((uint64_t)(uint32_t)(q[1] + 65536) << 17) |
                  ((uint64_t)(uint32_t)(q[2] + 65536) << 34) | ((uint64_t)(uint32_t)(lp + 16) << 51) |
                  ((uint64_t)code << 56);
            home = home_of(key, a.mask);
            fp = fingerprint_of(key);
            flags = 0;
        } else {
            flags = PF_V_KEYRANGE;
        }
    }
    key_out[i] = key;
    flags_out[i] = flags;
    if (fp_out) fp_out[i] = fp;
    if (home_out) home_out[i] = home;
}

hipError_t launch_build_keys(const float *px, const float *py, const float *pz, const float *nx, const float *ny,
                             const float *nz, const uint8_t *valid, uint32_t n, const KeyArgs &a, uint64_t *key,
                             uint32_t *fp, uint32_t *home, uint8_t *flags, hipStream_t st) {
    const uint32_t blocks = (n + kBlock - 1) / kBlock;
    build_keys_kernel<<<blocks, kBlock, 0, st>>>(px, py, pz, nx, ny, nz, valid, n, a, key, fp, home, flags);
    return hipGetLastError();
}

}  // namespace pfk
