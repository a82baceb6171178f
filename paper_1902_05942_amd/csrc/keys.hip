// Key construction (Algorithm 1) for gfx950: one vertex per lane, coalesced
// structure-of-arrays streams in (positions and normals of valid vertices
// only), 8-byte keys and 1-byte flags out.
#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

__global__ __launch_bounds__(kBlock) void build_keys_kernel(
    const float *__restrict__ px, const float *__restrict__ py, const float *__restrict__ pz,
    const float *__restrict__ nx, const float *__restrict__ ny, const float *__restrict__ nz,
    const uint8_t *__restrict__ valid, uint32_t n, KeyArgs a, uint64_t *__restrict__ key_out,
    uint32_t *__restrict__ fp_out, uint32_t *__restrict__ home_out, uint8_t *__restrict__ flags_out) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const PcgJump jp(a.seed, a.idx_base);
    uint64_t key = 0;
    uint32_t fp = 0, home = 0;
    uint8_t flags = PF_V_INVALID;
    if (valid == nullptr || valid[i] != 0) {  // masked vertices read nothing more
        const float x[3] = {px[i], py[i], pz[i]};
        const float nr[3] = {nx[i], ny[i], nz[i]};
        flags = vertex_key(x, nr, true, a.cam, a.s, a.inv_s, jp, i, a.mask, key, fp, home);
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
