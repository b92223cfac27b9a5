// Image pyramid at scale 1.2 (Sec. III-2): level l is resampled from level
// l-1 by bilinear interpolation at half-pixel centres.  Source coordinates
// are floored to Q8, the four 8-bit weights give a Q16 sum rounded half up:
//   ((256-fx)(256-fy) p_aa + fx (256-fy) p_ab + (256-fx) fy p_ba + fx fy p_bb
//    + 32768) >> 16,
// evaluated here as a horizontal then a vertical integer lerp (the same
// exact sum, factored: h = 256 a + fx (b - a), v = 256 h0 + fy (h1 - h0)).
//
// One launch per level covers that level of every image.  A block writes a
// 128 x 32 output tile: it stages the source window (chosen on the host, at
// most 256 x 44 bytes) in LDS with 16-byte loads, reads per-column and per-
// row source indices and weights from host-built tables (no division on the
// device), and each thread produces a 4 x 4 block of outputs.  Output rows
// of a block share source rows, so each needed source row is lerped
// horizontally once per column; results are stored as 32-bit words.
#include "vsfe_internal.h"

namespace vsfe {

constexpr int PYR_LDS_W = PYR_SW + 16;  // padded row stride (bank spread), 16-byte aligned
constexpr int PYR_TASKS = (PYR_SH * (PYR_SW / 16) + 255) / 256;

// 16 consecutive bytes of a row from x, coordinates clamped to [0, w).
__device__ __forceinline__ uint4 fetch16c(const uint8_t *row, int x, int w, bool aligned) {
    if (aligned && x >= 0 && x + 15 < w) return *(const uint4 *)(row + x);
    uint32_t v[4] = {0, 0, 0, 0};
    for (int j = 0; j < 16; j++) v[j >> 2] |= (uint32_t)row[min(max(x + j, 0), w - 1)] << (8 * (j & 3));
    return make_uint4(v[0], v[1], v[2], v[3]);
}

__global__ __launch_bounds__(256) void pyramid_level_kernel(const ImageDev *__restrict__ imgs,
                                                            const PyrItem *__restrict__ items, int level,
                                                            const uint32_t *__restrict__ coord,
                                                            const uint8_t *__restrict__ images,
                                                            uint8_t *__restrict__ pyr, int aligned0) {
    __shared__ __attribute__((aligned(16))) uint32_t s_src[PYR_SH * (PYR_LDS_W / 4)];
    const PyrItem it = items[xcd_item(blockIdx.x, gridDim.x)];
    const LevelDev s = imgs[it.image].lv[level - 1];
    const LevelDev d = imgs[it.image].lv[level];
    const uint8_t *src = (level == 1 ? images : pyr) + s.offset;
    uint8_t *dst = pyr + d.offset;
    const int tid = threadIdx.x;
    const bool aligned = level > 1 || aligned0;

    // stage rows ys .. ys+nrows-1, columns xs .. xs+ncols-1 (clamped to the
    // level) as 16-byte chunks; all of a thread's loads are issued before any
    // LDS store so they are in flight together
    const int cpr = it.ncols >> 4;
    const int ntask = it.nrows * cpr;
    uint4 v[PYR_TASKS];
    int at[PYR_TASKS];
#pragma unroll
    for (int u = 0; u < PYR_TASKS; u++) {
        const int q = tid + 256 * u;
        at[u] = -1;
        if (q < ntask) {
            const int rr = q / cpr, k = q - rr * cpr;
            const int gy = min((int)it.ys + rr, s.h - 1);
            v[u] = fetch16c(src + (int64_t)gy * s.pitch, (int)it.xs + 16 * k, s.w, aligned);
            at[u] = rr * (PYR_LDS_W / 16) + k;
        }
    }
#pragma unroll
    for (int u = 0; u < PYR_TASKS; u++)
        if (at[u] >= 0) ((uint4 *)s_src)[at[u]] = v[u];
    __syncthreads();

    const uint8_t *sb = (const uint8_t *)s_src;
    const int ox = it.tx * PYR_TW + (tid & 31) * 4;
    const int oy0 = it.ty * PYR_TH + (tid >> 5) * 4;
    if (ox >= d.w || oy0 >= d.h) return;
    int xa[4], fx[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t e = coord[d.xtab + min(ox + j, d.w - 1)];
        xa[j] = (int)(e & 0xFFFFu) - (int)it.xs;
        fx[j] = (int)(e >> 16);
    }
    // horizontal lerp of source row `ya` (LDS-local) for the 4 columns
    auto hrow = [&](int ya, int *h) {
        const uint8_t *r = sb + ya * PYR_LDS_W;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int a = r[xa[j]], b = r[xa[j] + 1];
            h[j] = (a << 8) + fx[j] * (b - a);
        }
    };
    int cur_row = -1;
    int h0[4], h1[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int oy = oy0 + k;
        if (oy >= d.h) break;
        const uint32_t e = coord[d.ytab + oy];
        const int ya = (int)(e & 0xFFFFu) - (int)it.ys, fy = (int)(e >> 16);
        if (ya == cur_row + 1 && cur_row >= 0) {
#pragma unroll
            for (int j = 0; j < 4; j++) h0[j] = h1[j];
            hrow(ya + 1, h1);
        } else if (ya != cur_row) {
            hrow(ya, h0);
            hrow(ya + 1, h1);
        }
        cur_row = ya;
        uint32_t word = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int v = ((h0[j] << 8) + fy * (h1[j] - h0[j]) + 32768) >> 16;
            word |= (uint32_t)v << (8 * j);
        }
        uint8_t *out = dst + (int64_t)oy * d.pitch + ox;
        if (ox + 3 < d.w) {
            *(uint32_t *)out = word;
        } else {
            for (int j = 0; ox + j < d.w; j++) out[j] = (uint8_t)(word >> (8 * j));
        }
    }
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t pyramid_build(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                 uint8_t *pyr, int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !pyr) return fail(VSFE_EINVAL, "null image or pyramid buffer");
    const int aligned = b->aligned_input16 && (((uintptr_t)images & 15) == 0) ? 1 : 0;
    hipStream_t st = (hipStream_t)stream;
    for (int l = 1; l < b->info.n_levels; l++) {
        const int n = b->pyr_start[l + 1] - b->pyr_start[l];
        if (n <= 0) continue;
        hipLaunchKernelGGL(pyramid_level_kernel, dim3(n), dim3(256), 0, st, b->d_images,
                           b->d_pyr_items + b->pyr_start[l], l, b->d_coord, images, pyr, aligned);
        rc = check_launch("pyramid_build");
        if (rc) return rc;
    }
    return VSFE_OK;
}
