// Pixel resolve (Section 3) for gfx950: after filtering, each selected
// vertex's value is multiplied by its throughput (the attenuation from the
// camera along its path up to the vertex) and accumulated in its pixel.
// Vertices are bounce-major (vertex b of pixel p at b * pixels + p), so one
// lane per pixel reads the path's vertices with coalesced loads, one bounce
// after the other; per channel acc = acc + t * c in binary32, bounce 0
// first, over the vertices with valid != 0.
#include "pf_kernels.h"
#include "pf_ops.h"

namespace pfk {

__global__ __launch_bounds__(kBlock) void resolve_kernel(const float *__restrict__ r, const float *__restrict__ g,
                                                         const float *__restrict__ b, const float *__restrict__ tr,
                                                         const float *__restrict__ tg, const float *__restrict__ tb,
                                                         const uint8_t *__restrict__ valid, uint32_t pixels,
                                                         uint32_t verts, bool accumulate, float *pr, float *pg,
                                                         float *pb) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= pixels) return;
    float a0 = accumulate ? pr[p] : 0.0f, a1 = accumulate ? pg[p] : 0.0f, a2 = accumulate ? pb[p] : 0.0f;
    for (uint32_t k = 0; k < verts; ++k) {
        const size_t v = (size_t)k * pixels + p;
        if (valid && valid[v] == 0) continue;
        const float t0 = tr ? tr[v] : 1.0f, t1 = tg ? tg[v] : 1.0f, t2 = tb ? tb[v] : 1.0f;
        const float m0 = t0 * r[v], m1 = t1 * g[v], m2 = t2 * b[v];
        a0 = a0 + m0;
        a1 = a1 + m1;
        a2 = a2 + m2;
    }
    pr[p] = a0;
    pg[p] = a1;
    pb[p] = a2;
}

hipError_t launch_resolve(const float *r, const float *g, const float *b, const float *tr, const float *tg,
                          const float *tb, const uint8_t *valid, uint32_t pixels, uint32_t verts, bool accumulate,
                          float *pr, float *pg, float *pb, hipStream_t st) {
    const uint32_t blocks = (pixels + kBlock - 1) / kBlock;
    resolve_kernel<<<blocks, kBlock, 0, st>>>(r, g, b, tr, tg, tb, valid, pixels, verts, accumulate, pr, pg, pb);
    return hipGetLastError();
}

}  // namespace pfk
