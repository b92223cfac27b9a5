// Sub-pixel stereo refinement by correlation minimisation (the middle-end's
// stereo matcher pairs correlation minimisation with descriptor-distance
// minimisation, Sec. III-3 and Fig. "slampipeline").
//
// For a left keypoint with an accepted descriptor match, on the keypoint's
// pyramid level (unsmoothed): SAD(s) over the (2w+1)^2 window around the
// left keypoint against the window around the matched right column shifted
// by s in [-r, r] (same rows: the pair is rectified); s* = least SAD (ties:
// smaller |s|, then smaller s); not refined when there is no match, a
// window leaves the level or s* = +-r; otherwise the vertex of the parabola
// through SAD(s* - 1), SAD(s*), SAD(s* + 1), offset (S- - S+) /
// (2 (S- - 2 S0 + S+)) in 1/256 pixel rounded half away from zero, and the
// native-scale disparity floor(((256 xl - (256 (xr + s*) + offset)) S_l +
// 2^15) / 2^16) in 1/256 pixel.
//
// GPU mapping: a group of 16 lanes per left keypoint slot (4 per wave);
// lane k of the group takes window row k.  It loads the row's window bytes
// of the left view and the right view's span of 2 (w + r) + 1 bytes as
// aligned dwords once, re-bases the span to every byte offset with
// v_alignbyte, and accumulates |a - b| four bytes per v_sad_u8 for every
// shift.  The per-row SADs are summed over the group by recursive halving
// (four exchange steps, 8 + 4 + 2 + 1 shuffles), which leaves the SAD of
// shift index k in lane k.  A 16-lane minimum of (SAD, |s|, s) picks s*;
// the two neighbouring SADs come from their lanes; the group's first lane
// fits the parabola.
#include <limits.h>

#include "vsfe_internal.h"

namespace vsfe {

constexpr int RF_GROUP = 16;             // lanes per keypoint: window rows 2 w + 1 and shifts 2 r + 1 <= 15
constexpr int RF_MAX_W = 7, RF_MAX_R = 7;

struct RefineArgs {
    int32_t scale_q16[VSFE_MAX_LEVELS];
    int n_max, n_pairs, w, r, aligned0;
};

// Aligned dword at byte offset `at` of a row (zero if it starts at or past
// the row's end `w`): with 4-byte aligned rows and a pitch that is a
// multiple of 4, a dword that starts inside the row ends inside its pitch.
__device__ __forceinline__ uint32_t row_dword(const uint8_t *row, int at, int w, bool aligned) {
    if (at >= w) return 0u;
    if (aligned) return *(const uint32_t *)(row + at);
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < 4; b++)
        if (at + b < w) v |= (uint32_t)row[at + b] << (8 * b);
    return v;
}

// The n = 2 w + 1 window bytes of a row starting at column x0 as up to four
// words (bytes past n zero): aligned dwords from (x0 & ~3), shifted into
// place by the byte offset.
__device__ __forceinline__ void window_words(const uint8_t *row, int x0, int wl, bool aligned, int nb, uint32_t *out) {
    const int a = x0 & ~3, sh = x0 & 3;
    uint32_t d[5];
#pragma unroll
    for (int k = 0; k < 5; k++) d[k] = row_dword(row, a + 4 * k, wl, aligned);
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const uint32_t v = __builtin_amdgcn_alignbyte(d[k + 1], d[k], (uint32_t)sh);
        const int left = nb - 4 * k;                      // window bytes still to place
        out[k] = left >= 4 ? v : (left <= 0 ? 0u : (v & ((1u << (8 * left)) - 1u)));
    }
}

__global__ __launch_bounds__(256) void refine_kernel(const ImageDev *__restrict__ imgs, vsfe_kp_soa kps,
                                                     const int32_t *__restrict__ kp_count,
                                                     const int32_t *__restrict__ midx, const uint8_t *__restrict__ images,
                                                     const uint8_t *__restrict__ pyr, int32_t *__restrict__ disp,
                                                     uint32_t *__restrict__ sad_out, RefineArgs a) {
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / RF_GROUP;
    const int k = threadIdx.x & (RF_GROUP - 1);
    const int pair = (int)(grp / a.n_max);
    const int i = (int)(grp - (int64_t)pair * a.n_max);
    if (pair >= a.n_pairs) return;                        // (whole groups exit together)
    const int li = 2 * pair, ri = 2 * pair + 1;
    if (i >= kp_count[li]) return;
    const int64_t o = (int64_t)pair * a.n_max + i;
    const int j = midx[o];
    const ImageDev &iml = imgs[li];
    const int64_t ls = iml.kp_offset + i;
    const int level = min((int)kps.level[ls], iml.n_levels - 1);
    const LevelDev lv = iml.lv[level];
    const int xl = kps.x[ls], yl = kps.y[ls];
    const int w = a.w, r = a.r, nb = 2 * w + 1;
    int xr = 0;
    bool ok = j >= 0 && j < kp_count[ri];
    if (ok) xr = kps.x[imgs[ri].kp_offset + j];
    ok = ok && xl - w >= 0 && xl + w < lv.w && yl - w >= 0 && yl + w < lv.h && xr - r - w >= 0 && xr + r + w < lv.w;
    if (!ok) {                                            // uniform over the group
        if (k == 0) {
            disp[o] = INT_MIN;
            if (sad_out) sad_out[o] = 0xFFFFFFFFu;
        }
        return;
    }
    const bool aligned = level > 0 || a.aligned0 != 0;
    const uint8_t *basel = (level == 0 ? images : pyr) + iml.lv[level].offset;
    const uint8_t *baser = (level == 0 ? images : pyr) + imgs[ri].lv[level].offset;
    // col[t]: this lane's window row, SAD at shift s = t - r
    uint32_t col[RF_GROUP];
#pragma unroll
    for (int t = 0; t < RF_GROUP; t++) col[t] = 0;
    if (k < nb) {
        const int64_t ro = (int64_t)(yl + k - w) * lv.pitch;
        uint32_t lw[4];
        window_words(basel + ro, xl - w, lv.w, aligned, nb, lw);
        // the right row's span xr - r - w .. xr + r + w, re-based to byte 0
        // (e0) and to bytes 1..3 (e1..e3): the window at shift index t is
        // the four words from byte t of the span
        const int x0 = xr - r - w, need = (x0 & 3) + nb + 2 * r;
        const int sh = x0 & 3;
        uint32_t d[9];
#pragma unroll
        for (int q = 0; q < 9; q++) d[q] = 4 * q < need ? row_dword(baser + ro, (x0 & ~3) + 4 * q, lv.w, aligned) : 0u;
        uint32_t e[4][8];
#pragma unroll
        for (int q = 0; q < 8; q++) e[0][q] = __builtin_amdgcn_alignbyte(d[q + 1], d[q], (uint32_t)sh);
#pragma unroll
        for (int u = 1; u < 4; u++)
#pragma unroll
            for (int q = 0; q < 7; q++) e[u][q] = __builtin_amdgcn_alignbyte(e[0][q + 1], e[0][q], (uint32_t)u);
        uint32_t m[4];                                    // window bytes of each word
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int left = nb - 4 * q;
            m[q] = left >= 4 ? 0xFFFFFFFFu : (left <= 0 ? 0u : (1u << (8 * left)) - 1u);
        }
#pragma unroll
        for (int t = 0; t < 2 * RF_MAX_R + 1; t++) {
            const int q = t >> 2, u = t & 3;
            uint32_t acc = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) acc = __builtin_amdgcn_sad_u8(lw[j], e[u][q + j] & m[j], acc);
            col[t] = t <= 2 * r ? acc : 0u;
        }
    }
    // column sums over the group's 16 rows by recursive halving: after the
    // step that exchanges with lane k ^ h, lane k holds the partial sums of
    // the shift indices whose bit h matches its own, so lane k ends with the
    // full SAD of shift index k
#pragma unroll
    for (int h = RF_GROUP / 2; h > 0; h >>= 1) {
        const bool up = (k & h) != 0;
#pragma unroll
        for (int j = 0; j < h; j++) {
            const uint32_t keep = up ? col[j + h] : col[j];
            const uint32_t give = up ? col[j] : col[j + h];
            col[j] = keep + (uint32_t)__shfl_xor((int)give, h, RF_GROUP);
        }
    }
    const uint32_t acc = col[0];
    const int s = k - r;
    const bool active = k <= 2 * r;
    // least (SAD, |s|, s) over the group: SAD < 2^16 (15 x 15 x 255), |s|, s + 8 in a byte each
    const uint32_t as = (uint32_t)(s < 0 ? -s : s);
    uint32_t key = active ? (acc << 16) | (as << 8) | (uint32_t)(s + 8) : 0xFFFFFFFFu;
#pragma unroll
    for (int d = RF_GROUP / 2; d > 0; d >>= 1) key = min(key, (uint32_t)__shfl_xor((int)key, d, RF_GROUP));
    const int sb = (int)(key & 0xFFu) - 8;
    const int base_lane = (threadIdx.x & 63) & ~(RF_GROUP - 1);
    const uint32_t sm = (uint32_t)__shfl((int)acc, base_lane + (sb - 1 + r), 64);
    const uint32_t sp = (uint32_t)__shfl((int)acc, base_lane + (sb + 1 + r), 64);
    if (k != 0) return;
    if (sb == -r || sb == r) {
        disp[o] = INT_MIN;
        if (sad_out) sad_out[o] = 0xFFFFFFFFu;
        return;
    }
    const int s0 = (int)(key >> 16);
    const int den = (int)sm - 2 * s0 + (int)sp;           // >= 0: S0 is the least
    int off = 0;
    if (den != 0) {
        const int num = 128 * ((int)sm - (int)sp);        // |num| <= 128 den
        const int mag = num < 0 ? -num : num;
        const int q = (2 * mag + den) / (2 * den);
        off = num < 0 ? -q : q;
    }
    const int64_t d_level = 256 * (int64_t)xl - (256 * (int64_t)(xr + sb) + off);
    const int64_t v = d_level * a.scale_q16[level] + 32768;
    disp[o] = (int32_t)(v >> 16);                         // arithmetic shift: floor
    if (sad_out) sad_out[o] = (uint32_t)s0;
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t stereo_refine(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images, const uint8_t *pyr,
                                 const vsfe_kp_soa *kps, const int32_t *kp_count, const int32_t *match_idx,
                                 int32_t half_window, int32_t search_radius, int32_t *disp_q8, uint32_t *sad_min,
                                 int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !kps || !kp_count || !match_idx || !disp_q8 || (!pyr && b->info.n_levels > 1))
        return fail(VSFE_EINVAL, "null buffer");
    if (!kps->x || !kps->y || !kps->level) return fail(VSFE_EINVAL, "null keypoint array");
    if (!b->pairs_ok) return fail(VSFE_EINVAL, "stereo_refine needs pairs of equal-size images (2i, 2i+1)");
    if (half_window < 1 || half_window > RF_MAX_W) return fail(VSFE_EINVAL, "half_window out of 1..7");
    if (search_radius < 1 || search_radius > RF_MAX_R) return fail(VSFE_EINVAL, "search_radius out of 1..7");
    RefineArgs a;
    for (int l = 0; l < VSFE_MAX_LEVELS; l++) a.scale_q16[l] = ctx->scale_q16[l];
    a.n_max = ctx->p.n_max;
    a.n_pairs = b->n_images / 2;
    a.w = half_window;
    a.r = search_radius;
    a.aligned0 = b->aligned_input && (((uintptr_t)images & 3) == 0) ? 1 : 0;
    const int64_t groups = (int64_t)a.n_pairs * a.n_max;
    if (groups <= 0) return VSFE_OK;
    const int64_t blocks = (groups * RF_GROUP + 255) / 256;
    if (blocks >= ((int64_t)1 << 31)) return fail(VSFE_ECAPACITY, "too many keypoint slots");
    hipLaunchKernelGGL(refine_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, b->d_images, *kps,
                       kp_count, match_idx, images, pyr, disp_q8, sad_min, a);
    return check_launch("stereo_refine");
}
