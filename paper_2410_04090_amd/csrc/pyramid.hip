// Image pyramid at scale 1.2 (Sec. III-2): level l is resampled from level
// l-1 by bilinear interpolation at half-pixel centres.  Source coordinates
// are floored to Q8, the four 8-bit weights give a Q16 sum rounded half up:
//   ((256-fx)(256-fy) p_aa + fx (256-fy) p_ab + (256-fx) fy p_ba + fx fy p_bb
//    + 32768) >> 16,
// evaluated here as a horizontal then a vertical integer lerp (the same
// exact sum, factored: h = 256 a + fx (b - a), v = 256 h0 + fy (h1 - h0)).
//
// One launch per level covers that level of every image.  A block writes a
// 256 x 32 output tile: it stages the source window (chosen on the host, at
// most 336 x 44 bytes) in LDS with 16-byte loads and reads per-column and
// per-row source indices and weights from host-built tables (no division on
// the device).  Each lane produces 4 columns of its wave's 8 rows, so the
// source rows are uniform per wave: every needed source row is lerped
// horizontally once, two columns per packed 16-bit multiply-add
// (a (256 - fx) + b fx <= 65280 fits), with the 4 source bytes of a column
// pair gathered by one v_perm from two LDS dwords; the vertical lerp is a
// 32-bit multiply-add per output whose byte 2 is the rounded result, and the
// 4 outputs are stored as one 32-bit word.
#include "vsfe_internal.h"

namespace vsfe {

constexpr int PYR_LDS_W = PYR_SW + 16;  // padded row stride (bank spread), 16-byte aligned
constexpr int PYR_TASKS = (PYR_SH * (PYR_SW / 16) + 255) / 256;

typedef unsigned short pu2 __attribute__((ext_vector_type(2)));

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
    const struct { int w, h, pitch; int64_t offset; } s = {it.sw, it.sh, it.spitch, it.src_offset};
    const struct { int w, h, pitch, xtab, ytab; int64_t offset; } d = {it.dw, it.dh, it.dpitch, it.xtab, it.ytab,
                                                                      it.dst_offset};
    const uint8_t *src = (level == 1 ? images : pyr) + s.offset;
    uint8_t *dst = pyr + d.offset;
    const int tid = threadIdx.x;
    const bool aligned = level > 1 || aligned0;

    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    constexpr int ROWS = PYR_TH / 4;                     // output rows per wave
    const int oy0 = it.ty * PYR_TH + ROWS * wave;        // uniform
    const int ox = it.tx * PYR_TW + 4 * lane;
    // resampling table entries of the lane's 4 columns and the wave's rows,
    // loaded together with the staged rows
    uint32_t ex[4], ey[ROWS];
#pragma unroll
    for (int j = 0; j < 4; j++) ex[j] = coord[d.xtab + min(ox + j, d.w - 1)];
#pragma unroll
    for (int k = 0; k < ROWS; k++) ey[k] = coord[d.ytab + min(oy0 + k, d.h - 1)];

    // stage rows ys .. ys+nrows-1, columns xs .. xs+ncols-1 (clamped to the
    // level) as 16-byte chunks, task q = row q / 21, chunk q % 21 (a
    // constant divisor); all of a thread's loads are issued before any LDS
    // store so they are in flight together
    constexpr int CPR = PYR_SW / 16;
    uint4 v[PYR_TASKS];
    int at[PYR_TASKS];
#pragma unroll
    for (int u = 0; u < PYR_TASKS; u++) {
        const int q = tid + 256 * u;
        const int rr = q / CPR, k = q - rr * CPR;
        at[u] = -1;
        if (rr < it.nrows && 16 * k < it.ncols) {
            const int gy = min(it.ys + rr, s.h - 1);
            v[u] = fetch16c(src + (int64_t)gy * s.pitch, it.xs + 16 * k, s.w, aligned);
            at[u] = rr * (PYR_LDS_W / 16) + k;
        }
    }
#pragma unroll
    for (int u = 0; u < PYR_TASKS; u++)
        if (at[u] >= 0) ((uint4 *)s_src)[at[u]] = v[u];
    __syncthreads();

    if (oy0 >= d.h) return;
    // columns: source index (window-local) and weight of the lane's 4 outputs
    int o[4], fx[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        o[j] = (int)(ex[j] & 0xFFFFu) - it.xs;
        fx[j] = (int)(ex[j] >> 16);
    }
    // byte selectors of (a0, a1), (b0, b1), (a2, a3), (b2, b3) within the
    // two dwords at base01 / base23 (0x0c selects a zero byte)
    const int base01 = o[0] & ~3, base23 = o[2] & ~3;
    const uint32_t selA01 = (uint32_t)(o[0] - base01) | 0x0C00u | ((uint32_t)(o[1] - base01) << 16) | 0x0C000000u;
    const uint32_t selA23 = (uint32_t)(o[2] - base23) | 0x0C00u | ((uint32_t)(o[3] - base23) << 16) | 0x0C000000u;
    const uint32_t selB01 = selA01 + 0x00010001u, selB23 = selA23 + 0x00010001u;
    const pu2 W01 = {(unsigned short)(256 - fx[0]), (unsigned short)(256 - fx[1])};
    const pu2 W23 = {(unsigned short)(256 - fx[2]), (unsigned short)(256 - fx[3])};
    const pu2 F01 = {(unsigned short)fx[0], (unsigned short)fx[1]};
    const pu2 F23 = {(unsigned short)fx[2], (unsigned short)fx[3]};
    const uint8_t *sb = (const uint8_t *)s_src;
    // horizontal lerps (x 256) of window row ya for the 4 columns, as two u16 pairs
    auto hrow = [&](int ya, pu2 &h01, pu2 &h23) {
        const uint8_t *r = sb + ya * PYR_LDS_W;
        const uint32_t d0 = *(const uint32_t *)(r + base01), d1 = *(const uint32_t *)(r + base01 + 4);
        const uint32_t e0 = *(const uint32_t *)(r + base23), e1 = *(const uint32_t *)(r + base23 + 4);
        const pu2 A01 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(d1, d0, selA01));
        const pu2 B01 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(d1, d0, selB01));
        const pu2 A23 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(e1, e0, selA23));
        const pu2 B23 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(e1, e0, selB23));
        h01 = A01 * W01 + B01 * F01;
        h23 = A23 * W23 + B23 * F23;
    };
    uint8_t *out = dst + (int64_t)oy0 * d.pitch + ox;
    int cur = -2;
    pu2 t01, t23, u01, u23;                              // rows cur, cur + 1
#pragma unroll
    for (int k = 0; k < ROWS; k++) {
        const int oy = oy0 + k;
        if (oy >= d.h) break;                            // uniform
        const uint32_t e = ey[k];
        const int ya = (int)(e & 0xFFFFu) - it.ys;
        const uint32_t fy = e >> 16, wy = 256u - fy;
        if (ya == cur + 1) {                             // slide by one row
            t01 = u01;
            t23 = u23;
            hrow(ya + 1, u01, u23);
        } else if (ya != cur) {
            hrow(ya, t01, t23);
            hrow(ya + 1, u01, u23);
        }
        cur = ya;
        // (h0 (256 - fy) + h1 fy + 2^15) >> 16 is byte 2 of the sum
        const uint32_t s0 = (uint32_t)t01.x * wy + (uint32_t)u01.x * fy + 32768u;
        const uint32_t s1 = (uint32_t)t01.y * wy + (uint32_t)u01.y * fy + 32768u;
        const uint32_t s2 = (uint32_t)t23.x * wy + (uint32_t)u23.x * fy + 32768u;
        const uint32_t s3 = (uint32_t)t23.y * wy + (uint32_t)u23.y * fy + 32768u;
        const uint32_t word = __builtin_amdgcn_perm(s1, s0, 0x0C0C0602u) | (__builtin_amdgcn_perm(s3, s2, 0x0C0C0602u) << 16);
        if (ox + 3 < d.w) {
            *(uint32_t *)out = word;
        } else {
            for (int j = 0; ox + j < d.w; j++) out[j] = (uint8_t)(word >> (8 * j));
        }
        out += d.pitch;
    }
}

}  // namespace vsfe

using namespace vsfe;

static int32_t build_range(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images, uint8_t *pyr,
                           int32_t *status, int lb, int le, hipStream_t st) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !pyr) return fail(VSFE_EINVAL, "null image or pyramid buffer");
    const int aligned = b->aligned_input16 && (((uintptr_t)images & 15) == 0) ? 1 : 0;
    for (int l = lb; l < le; l++) {
        const int n = b->pyr_start[l + 1] - b->pyr_start[l];
        if (n <= 0) continue;
        hipLaunchKernelGGL(pyramid_level_kernel, dim3(n), dim3(256), 0, st, b->d_images,
                           b->d_pyr_items + b->pyr_start[l], l, b->d_coord, images, pyr, aligned);
        rc = check_launch("pyramid_build");
        if (rc) return rc;
    }
    return VSFE_OK;
}

extern "C" int32_t pyramid_build(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                 uint8_t *pyr, int32_t *status, void *stream) {
    if (!b) return fail(VSFE_EINVAL, "null batch");
    return build_range(ctx, b, images, pyr, status, 1, b->info.n_levels, (hipStream_t)stream);
}

extern "C" int32_t pyramid_build_levels(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                        uint8_t *pyr, int32_t level_begin, int32_t level_end, int32_t *status,
                                        void *stream) {
    if (!b) return fail(VSFE_EINVAL, "null batch");
    if (level_begin < 1 || level_end > b->info.n_levels || level_begin >= level_end)
        return fail(VSFE_EINVAL, "level range out of 1..n_levels or empty");
    return build_range(ctx, b, images, pyr, status, level_begin, level_end, (hipStream_t)stream);
}
