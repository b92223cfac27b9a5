// Feature Culling over a materialised response matrix, the way the paper
// schedules it (Sec. II-C-1), kept as an ablation beside the fused culling
// of fast_br_detect (which never writes the response matrix).
//
// Every scheme computes, per cell of side c, the largest key
// (response << 10) | (1023 - offset in cell) over the cell's pixels with a
// non-zero response: the strongest corner, ties to the first in raster
// order (0 = no corner), the same keys as fast_br_detect without a fallback
// threshold.
//
//  * MLPT + TEWA (scheme 0): vertical culling with N_t = ceil(c / n_loc)
//    threads per column, each taking n_loc consecutive rows (coalesced: the
//    lanes of a wave read consecutive columns), the first thread of each
//    column reducing the N_t partial maxima; horizontal culling with
//    ceil(c / n_loc) threads per cell reading the column maxima at a stride
//    of ceil(c / n_loc); the block is 128 threads wide in x and packs
//    floor(128 / c) cells side by side (thread-efficient warp allocation),
//    N_t threads high.
//  * log2 reduction (scheme 1): one block per cell, one thread per pixel,
//    a tree reduction in ceil(log2(c^2)) halving steps.
//  * MLPT with one block per cell (scheme 2): as scheme 0, but each block
//    holds a single cell (c threads wide), the allocation TEWA replaces.
#include "vsfe_internal.h"

namespace vsfe {

struct FcArgs {
    int level, cell, n_loc, nt, cpb, n_images;
    int64_t stride;           // output keys per image
};

__device__ __forceinline__ uint32_t crf_key(const uint16_t *crf, const LevelDev &lv, int x, int y, int x0c, int y0c,
                                            int c) {
    const uint32_t v = crf[lv.crf_offset + (int64_t)y * lv.w + x];
    return v ? (v << 10) | (1023u - (uint32_t)((y - y0c) * c + (x - x0c))) : 0u;
}

// scheme 0 (TEWA, cpb cells per block) and scheme 2 (cpb = 1): block
// (128 or c) x nt threads; blockIdx.x = cell-column group, .y = cell row,
// .z = image
__global__ __launch_bounds__(1024) void fc_mlpt_kernel(const ImageDev *__restrict__ imgs,
                                                       const uint16_t *__restrict__ crf, uint32_t *__restrict__ keys,
                                                       FcArgs a) {
    __shared__ uint32_t s_v[8][128];
    __shared__ uint32_t s_col[128];
    const ImageDev &im = imgs[blockIdx.z];
    const LevelDev lv = im.lv[a.level];
    const int c = a.cell;
    const int ncx = (lv.w + c - 1) / c, ncy = (lv.h + c - 1) / c;
    const int cy = blockIdx.y;
    if (cy >= ncy) return;                               // uniform
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int k = tx / c, j = tx - k * c;                // cell in the block, column in the cell
    const int cx = blockIdx.x * a.cpb + k;
    const bool col_ok = k < a.cpb && cx < ncx && cx * c + j < lv.w;
    const int x = cx * c + j, y0c = cy * c, x0c = cx * c;
    // vertical culling: rows [ty n_loc, (ty + 1) n_loc) of the column
    uint32_t m = 0;
    if (col_ok) {
        const int yb = y0c + ty * a.n_loc, ye = min(min(yb + a.n_loc, y0c + c), lv.h);
        for (int y = yb; y < ye; y++) m = max(m, crf_key(crf, lv, x, y, x0c, y0c, c));
    }
    s_v[ty][tx] = m;
    __syncthreads();
    if (ty == 0) {
        uint32_t v = s_v[0][tx];
        for (int t = 1; t < a.nt; t++) v = max(v, s_v[t][tx]);
        s_col[tx] = v;
    }
    __syncthreads();
    // horizontal culling: ceil(c / n_loc) threads per cell, stride access
    const int nth = a.nt;                                // = ceil(c / n_loc)
    if (ty == 0 && k < a.cpb && j < nth) {
        uint32_t v = 0;
        for (int jj = j; jj < c; jj += nth) v = max(v, s_col[k * c + jj]);
        s_v[1][tx] = v;                                  // row 1 is free after the column pass
    }
    __syncthreads();
    if (ty == 0 && k < a.cpb && j == 0 && cx < ncx) {
        uint32_t v = 0;
        for (int t = 0; t < nth; t++) v = max(v, s_v[1][tx + t]);
        keys[(int64_t)blockIdx.z * a.stride + (int64_t)cy * ncx + cx] = v;
    }
}

// scheme 1: one block per cell, one thread per pixel, halving tree reduction
__global__ __launch_bounds__(1024) void fc_log2_kernel(const ImageDev *__restrict__ imgs,
                                                       const uint16_t *__restrict__ crf, uint32_t *__restrict__ keys,
                                                       FcArgs a) {
    __shared__ uint32_t s[1024];
    const ImageDev &im = imgs[blockIdx.z];
    const LevelDev lv = im.lv[a.level];
    const int c = a.cell;
    const int ncx = (lv.w + c - 1) / c, ncy = (lv.h + c - 1) / c;
    const int cx = blockIdx.x, cy = blockIdx.y;
    if (cx >= ncx || cy >= ncy) return;                  // uniform
    const int t = threadIdx.x;
    const int x = cx * c + t % c, y = cy * c + t / c;
    s[t] = (t < c * c && x < lv.w && y < lv.h) ? crf_key(crf, lv, x, y, cx * c, cy * c, c) : 0u;
    __syncthreads();
    for (int h = blockDim.x >> 1; h > 0; h >>= 1) {
        if (t < h) s[t] = max(s[t], s[t + h]);
        __syncthreads();
    }
    if (t == 0) keys[(int64_t)blockIdx.z * a.stride + (int64_t)cy * ncx + cx] = s[0];
}

static int64_t fc_stride(const vsfe_batch *b, int level, int cell, int *max_ncx, int *max_ncy) {
    int64_t m = 0;
    *max_ncx = *max_ncy = 0;
    for (int i = 0; i < b->n_images; i++) {
        const LevelDev &lv = b->images[i].lv[level];
        const int ncx = (lv.w + cell - 1) / cell, ncy = (lv.h + cell - 1) / cell;
        m = std::max<int64_t>(m, (int64_t)ncx * ncy);
        *max_ncx = std::max(*max_ncx, ncx);
        *max_ncy = std::max(*max_ncy, ncy);
    }
    return m;
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t vsfe_fc_cull_stride(const vsfe_batch *b, int32_t level, int32_t cell, int64_t *stride) {
    if (!b || !stride) return fail(VSFE_EINVAL, "null argument");
    if (level < 0 || level >= b->info.n_levels) return fail(VSFE_EINVAL, "level out of range");
    if (cell < 1 || cell > 32) return fail(VSFE_EINVAL, "cell out of 1..32");
    int mx, my;
    *stride = fc_stride(b, level, cell, &mx, &my);
    return VSFE_OK;
}

extern "C" int32_t fc_cull_crf(const vsfe_ctx *ctx, const vsfe_batch *b, const uint16_t *crf, int32_t level,
                               int32_t cell, int32_t scheme, int32_t n_loc, uint32_t *keys, int64_t keys_elems,
                               int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!crf || !keys) return fail(VSFE_EINVAL, "null buffer");
    if (level < 0 || level >= b->info.n_levels) return fail(VSFE_EINVAL, "level out of range");
    if (cell < 1 || cell > 32) return fail(VSFE_EINVAL, "cell out of 1..32");
    if (scheme < 0 || scheme > 2) return fail(VSFE_EINVAL, "scheme must be 0 (MLPT + TEWA), 1 (log2) or 2 (MLPT, block per cell)");
    FcArgs a;
    a.level = level;
    a.cell = cell;
    a.n_images = b->n_images;
    int mx, my;
    a.stride = fc_stride(b, level, cell, &mx, &my);
    if (b->n_images > 65535 || my > 65535) return fail(VSFE_ECAPACITY, "grid too large");
    // the output depends on (level, cell): its size is checked here, before
    // any launch, rather than trusted
    const int64_t need = (int64_t)b->n_images * a.stride;
    if (keys_elems < need)
        return fail(VSFE_ECAPACITY, "keys holds " + std::to_string((long long)keys_elems) + " entries; level " +
                                        std::to_string(level) + " with cell " + std::to_string(cell) + " needs " +
                                        std::to_string((long long)need) + " (n_images x vsfe_fc_cull_stride)");
    hipStream_t st = (hipStream_t)stream;
    if (scheme == 1) {
        a.n_loc = a.nt = a.cpb = 1;
        const int threads = ((cell * cell + 63) / 64) * 64;
        int p2 = 64;
        while (p2 < threads) p2 <<= 1;                   // power of two for the halving steps
        hipLaunchKernelGGL(fc_log2_kernel, dim3((unsigned)mx, (unsigned)my, (unsigned)b->n_images), dim3(p2), 0, st,
                           b->d_images, crf, keys, a);
        return check_launch("fc_cull_crf (log2)");
    }
    if (n_loc < 1 || n_loc > 32) return fail(VSFE_EINVAL, "n_loc out of 1..32");
    a.n_loc = n_loc;
    a.nt = (cell + n_loc - 1) / n_loc;
    if (a.nt > 8) return fail(VSFE_EINVAL, "ceil(cell / n_loc) must be at most 8");
    a.cpb = scheme == 0 ? std::max(1, 128 / cell) : 1;
    const int bx = scheme == 0 ? 128 : cell;
    const unsigned gx = (unsigned)((mx + a.cpb - 1) / a.cpb);
    hipLaunchKernelGGL(fc_mlpt_kernel, dim3(gx, (unsigned)my, (unsigned)b->n_images), dim3(bx, a.nt), 0, st,
                       b->d_images, crf, keys, a);
    return check_launch("fc_cull_crf (MLPT)");
}
