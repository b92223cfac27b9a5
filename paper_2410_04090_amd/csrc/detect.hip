// FAST with Bounded Rectification, corner response and Feature Culling,
// fused in one launch over every (image, level, cell tile).
//
//  * Labels (Sec. II-A, Eq. 1): bright if I_p > I_c + eps, dark if
//    I_p < I_c - eps, on the 16-pixel radius-3 ring; |I_p - I_c| = eps is
//    similar.
//  * Corner (Eq. 3): the longest cyclic bright or dark run N satisfies
//    p_min <= N <= p_max (p_max = 16 is plain FAST, Eq. 2).
//  * Response (Sec. III-1): sum over the ring of |I_c - I_p|.
//  * Feature Culling (Sec. II-C-1): per cell the largest key
//    (score << 10) | (1023 - offset in cell), i.e. the strongest corner and,
//    on ties, the first in raster order; a cell without an eps_hi corner
//    takes its best eps_lo corner and is flagged.
//
// GPU mapping: a 256-thread block owns a rectangle of whole cells of one
// level, stages it with a 3-pixel halo in LDS, and reduces keys per cell
// with LDS atomicMax (max is order independent, so the result is exact and
// deterministic).  Every pixel first tests the four compass pixels: any
// run of 9 or more contiguous ring pixels contains two adjacent compass
// pixels, so only candidates pay for the full ring test.  The paper's
// MLPT/TEWA schemes pack 32-lane warps; here the whole cell tile is one
// block and no thread count depends on the cell size.
#include "vsfe_internal.h"

namespace vsfe {

constexpr int DET_MAX_TW = 128, DET_MAX_TH = 64;
constexpr int DET_LDS_W = DET_MAX_TW + 6, DET_LDS_H = DET_MAX_TH + 6;
constexpr int DET_MAX_CELLS = 512;

struct DetParams {
    int eps_hi, eps_lo, p_min, p_max, border, prefilter, eps_min;
};

__constant__ int8_t c_ring_dx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
__constant__ int8_t c_ring_dy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

// true if the 16-bit ring mask holds a cyclic run of at least k ones (k <= 16)
__device__ __forceinline__ bool has_run(uint32_t m, int k) {
    const uint32_t x = m | (m << 16);
    uint32_t y = x;
    for (int s = 1; s < k; s++) y &= x >> s;
    return y != 0;
}

__device__ __forceinline__ bool br_corner(uint32_t m, int p_min, int p_max) {
    if (!has_run(m, p_min)) return false;
    return p_max >= 16 || !has_run(m, p_max + 1);
}

// Does level-l cell (cx, cy) overlap a kept level-0 cell?  Footprint at the
// native scale: [x S >> 16, ceil((x + c) S / 2^16)) with x = cx c, same in y.
__device__ __forceinline__ bool cell_runs(const uint8_t *mask0, const LevelDev &l0, const LevelDev &lv,
                                          int cx, int cy) {
    const int64_t S = lv.scale_q16, c = lv.cell, c0 = l0.cell;
    const int64_t fx0 = ((int64_t)cx * c * S) >> 16, fx1 = (((int64_t)cx * c + c) * S + 65535) >> 16;
    const int64_t fy0 = ((int64_t)cy * c * S) >> 16, fy1 = (((int64_t)cy * c + c) * S + 65535) >> 16;
    int a0 = (int)(fx0 / c0), a1 = (int)((fx1 - 1) / c0), b0 = (int)(fy0 / c0), b1 = (int)((fy1 - 1) / c0);
    a1 = a1 < l0.ncx - 1 ? a1 : l0.ncx - 1;
    b1 = b1 < l0.ncy - 1 ? b1 : l0.ncy - 1;
    for (int y = b0; y <= b1; y++)
        for (int x = a0; x <= a1; x++)
            if (mask0[y * l0.ncx + x]) return true;
    return false;
}

__global__ __launch_bounds__(256) void fast_br_kernel(const ImageDev *__restrict__ imgs,
                                                      const DetItem *__restrict__ items,
                                                      const uint8_t *__restrict__ images,
                                                      const uint8_t *__restrict__ pyr,
                                                      const uint8_t *__restrict__ mask,
                                                      uint32_t *__restrict__ cell_keys,
                                                      uint16_t *__restrict__ crf, DetParams prm) {
    __shared__ uint8_t tile[DET_LDS_H * DET_LDS_W];
    __shared__ uint32_t s_hi[DET_MAX_CELLS], s_lo[DET_MAX_CELLS];
    __shared__ uint8_t s_run[DET_MAX_CELLS];
    __shared__ int s_any;

    const DetItem it = items[blockIdx.x];
    const ImageDev &im = imgs[it.image];
    const LevelDev lv = im.lv[it.level];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int c = lv.cell;
    const int nk = it.nkx * it.nky;
    const int x0 = it.cx0 * c, y0 = it.cy0 * c;
    const int x1 = min(x0 + it.nkx * c, lv.w), y1 = min(y0 + it.nky * c, lv.h);
    const int tw = x1 - x0, th = y1 - y0;

    // learned gating: which cells of this tile run at all
    if (tid == 0) s_any = 0;
    __syncthreads();
    for (int k = tid; k < nk; k += 256) {
        bool run = true;
        if (mask) run = cell_runs(mask + im.cell0_offset, im.lv[0], lv, it.cx0 + k % it.nkx, it.cy0 + k / it.nkx);
        s_run[k] = run;
        s_hi[k] = 0;
        s_lo[k] = 0;
        if (run) s_any = 1;
    }
    __syncthreads();
    if (!s_any && !crf) {
        for (int k = tid; k < nk; k += 256)
            cell_keys[lv.cell_offset + (int64_t)(it.cy0 + k / it.nkx) * lv.ncx + (it.cx0 + k % it.nkx)] = 0;
        return;
    }

    // stage the tile and its 3-pixel halo
    const uint8_t *src = (it.level == 0 ? images : pyr) + lv.offset;
    const int hw = tw + 6, hh = th + 6;
    for (int r = ty; r < hh; r += 4) {
        const int gy = y0 - 3 + r;
        for (int q = tx; q < hw; q += 64) {
            const int gx = x0 - 3 + q;
            uint8_t v = 0;
            if (gx >= 0 && gx < lv.w && gy >= 0 && gy < lv.h) v = src[(int64_t)gy * lv.pitch + gx];
            tile[r * DET_LDS_W + q] = v;
        }
    }
    __syncthreads();

    const int B = prm.border;
    for (int ly = ty; ly < th; ly += 4) {
        const int gy = y0 + ly;
        for (int lx = tx; lx < tw; lx += 64) {
            const int gx = x0 + lx;
            const bool valid = gx >= B && gx < lv.w - B && gy >= B && gy < lv.h - B;
            uint16_t resp = 0;
            const uint8_t *t = &tile[(ly + 3) * DET_LDS_W + (lx + 3)];
            const int ctr = t[0];
            bool cand = valid;
            if (valid && prm.prefilter) {
                const int hi = ctr + prm.eps_min, lo = ctr - prm.eps_min;
                const int p0 = t[-3 * DET_LDS_W], p4 = t[3], p8 = t[3 * DET_LDS_W], p12 = t[-3];
                const bool b0 = p0 > hi, b4 = p4 > hi, b8 = p8 > hi, b12 = p12 > hi;
                const bool d0 = p0 < lo, d4 = p4 < lo, d8 = p8 < lo, d12 = p12 < lo;
                if (prm.prefilter == 2)
                    cand = (b0 && b4) || (b4 && b8) || (b8 && b12) || (b12 && b0) || (d0 && d4) || (d4 && d8) ||
                           (d8 && d12) || (d12 && d0);
                else
                    cand = b0 || b4 || b8 || b12 || d0 || d4 || d8 || d12;
            }
            if (cand) {
                int p[16];
#pragma unroll
                for (int k = 0; k < 16; k++) p[k] = t[c_ring_dy[k] * DET_LDS_W + c_ring_dx[k]];
                uint32_t bh = 0, dh = 0, bl = 0, dl = 0;
                int score = 0;
#pragma unroll
                for (int k = 0; k < 16; k++) {
                    bh |= (uint32_t)(p[k] > ctr + prm.eps_hi) << k;
                    dh |= (uint32_t)(p[k] < ctr - prm.eps_hi) << k;
                    bl |= (uint32_t)(p[k] > ctr + prm.eps_lo) << k;
                    dl |= (uint32_t)(p[k] < ctr - prm.eps_lo) << k;
                    score += abs(p[k] - ctr);
                }
                const bool c_hi = br_corner(bh, prm.p_min, prm.p_max) || br_corner(dh, prm.p_min, prm.p_max);
                const bool c_lo = prm.eps_lo >= 0 &&
                                  (br_corner(bl, prm.p_min, prm.p_max) || br_corner(dl, prm.p_min, prm.p_max));
                if (c_hi) resp = (uint16_t)score;
                if (c_hi || c_lo) {
                    const int kx = lx / c, ky = ly / c;
                    const int k = ky * it.nkx + kx;
                    const uint32_t off = (uint32_t)((ly - ky * c) * c + (lx - kx * c));
                    const uint32_t key = ((uint32_t)score << 10) | (1023u - off);
                    if (s_run[k]) {
                        if (c_hi) atomicMax(&s_hi[k], key);
                        if (c_lo) atomicMax(&s_lo[k], key);
                    }
                }
            }
            if (crf) crf[lv.crf_offset + (int64_t)gy * lv.w + gx] = resp;
        }
    }
    __syncthreads();
    for (int k = tid; k < nk; k += 256) {
        const uint32_t hi = s_hi[k], lo = s_lo[k];
        const uint32_t v = hi ? hi : (lo ? (lo | VSFE_KEY_FALLBACK) : 0u);
        cell_keys[lv.cell_offset + (int64_t)(it.cy0 + k / it.nkx) * lv.ncx + (it.cx0 + k % it.nkx)] = v;
    }
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t fast_br_detect(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                  const uint8_t *pyr, const uint8_t *cell_mask, uint32_t *cell_keys,
                                  uint16_t *crf_debug, int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !cell_keys || (!pyr && b->info.n_levels > 1)) return fail(VSFE_EINVAL, "null buffer");
    const vsfe_params &p = ctx->p;
    DetParams prm;
    prm.eps_hi = p.eps_hi;
    prm.eps_lo = p.eps_lo;
    prm.p_min = p.p_min;
    prm.p_max = p.p_max;
    prm.border = p.border;
    prm.eps_min = p.eps_lo >= 0 ? p.eps_lo : p.eps_hi;
    prm.prefilter = p.p_min >= 9 ? 2 : (p.p_min >= 5 ? 1 : 0);
    if (b->n_det_items <= 0) return VSFE_OK;
    hipLaunchKernelGGL(fast_br_kernel, dim3(b->n_det_items), dim3(256), 0, (hipStream_t)stream, b->d_images,
                       b->d_det_items, images, pyr, cell_mask, cell_keys, crf_debug, prm);
    return check_launch("fast_br_detect");
}
