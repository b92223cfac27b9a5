// Image pyramid at scale 1.2 (Sec. III-2): level l is resampled from level
// l-1 by bilinear interpolation at half-pixel centres.  Source coordinates
// are floored to Q8, the four 8-bit weights give a Q16 sum rounded half up.
//
// One launch per level covers that level of every image in the batch; a
// block writes a 64 x 16 output tile, each thread one column of 4 rows.
// The resampling is a gather of 4 neighbouring bytes of the previous level
// (L2-resident, just written), so the kernel is bound by memory latency and
// bytes, not arithmetic.
#include "vsfe_internal.h"

namespace vsfe {

// Q8 source coordinate of output o for a resize n_src -> n_dst:
// floor(((2 o + 1) n_src - n_dst) * 128 / n_dst), split into two 32-bit
// divisions so that the 34-bit product never forms.
__device__ __forceinline__ void q8_coord(uint32_t o, uint32_t n_src, uint32_t n_dst, int &a, int &b, int &f) {
    const uint32_t q = (2u * o + 1u) * n_src - n_dst;   // < 2 n_dst n_src < 2^27
    const uint32_t hi = q / n_dst, rem = q - hi * n_dst;
    const uint32_t t = hi * 128u + (rem * 128u) / n_dst;
    a = (int)(t >> 8);
    f = (int)(t & 255u);
    b = a + 1 < (int)n_src ? a + 1 : (int)n_src - 1;
}

__global__ __launch_bounds__(256) void pyramid_level_kernel(const ImageDev *__restrict__ imgs,
                                                            const PyrItem *__restrict__ items, int level,
                                                            const uint8_t *__restrict__ images,
                                                            uint8_t *__restrict__ pyr) {
    const PyrItem it = items[blockIdx.x];
    const LevelDev s = imgs[it.image].lv[level - 1];
    const LevelDev d = imgs[it.image].lv[level];
    const uint8_t *src = (level == 1 ? images : pyr) + s.offset;
    uint8_t *dst = pyr + d.offset;
    const int x = it.tx * PYR_TW + (threadIdx.x & (PYR_TW - 1));
    const int yb = it.ty * PYR_TH + (threadIdx.x / PYR_TW) * 4;
    if (x >= d.w) return;
    int xa, xb, fx;
    q8_coord((uint32_t)x, (uint32_t)s.w, (uint32_t)d.w, xa, xb, fx);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int y = yb + k;
        if (y >= d.h) break;
        int ya, ybb, fy;
        q8_coord((uint32_t)y, (uint32_t)s.h, (uint32_t)d.h, ya, ybb, fy);
        const uint8_t *ra = src + (int64_t)ya * s.pitch;
        const uint8_t *rb = src + (int64_t)ybb * s.pitch;
        const int v = (256 - fx) * (256 - fy) * ra[xa] + fx * (256 - fy) * ra[xb] +
                      (256 - fx) * fy * rb[xa] + fx * fy * rb[xb];
        dst[(int64_t)y * d.pitch + x] = (uint8_t)((v + 32768) >> 16);
    }
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t pyramid_build(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                 uint8_t *pyr, int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !pyr) return fail(VSFE_EINVAL, "null image or pyramid buffer");
    hipStream_t st = (hipStream_t)stream;
    for (int l = 1; l < b->info.n_levels; l++) {
        const int n = b->pyr_start[l + 1] - b->pyr_start[l];
        if (n <= 0) continue;
        hipLaunchKernelGGL(pyramid_level_kernel, dim3(n), dim3(256), 0, st, b->d_images,
                           b->d_pyr_items + b->pyr_start[l], l, images, pyr);
        rc = check_launch("pyramid_build");
        if (rc) return rc;
    }
    return VSFE_OK;
}
