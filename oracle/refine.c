/*
 * Oracle: sub-pixel stereo refinement by correlation minimisation (the
 * middle-end's stereo matcher of Sec. III-3 and Fig. "slampipeline"
 * pairs correlation minimisation with descriptor-distance minimisation),
 * test infrastructure only.
 *
 * The paper names the step without defining its measure, window or
 * sub-pixel rule; the reading taken here:
 *   - a left keypoint i with an accepted descriptor match j (same level l,
 *     level coordinates (xl, yl) and xr) is refined on level l of the
 *     unsmoothed pyramid;
 *   - SAD(s) = sum over dy, dx in [-w, w] of
 *       |L_l(xl + dx, yl + dy) - R_l(xr + s + dx, yl + dy)|,
 *     for every shift s in [-r, r] (rows of the left keypoint: the pair is
 *     rectified);
 *   - s* = the shift of least SAD, ties to the smaller |s|, then to the
 *     smaller s;
 *   - not refined when there is no match, when a window leaves the level,
 *     or when s* = -r or r (the minimum may lie outside the range);
 *   - otherwise the parabola through (s* - 1, S-), (s*, S0), (s* + 1, S+)
 *     has its vertex at s* + (S- - S+) / (2 (S- - 2 S0 + S+)) (offset 0 when
 *     the denominator is 0); the offset lies in [-1/2, 1/2] because S0 is
 *     the least of the three, and is taken in 1/256 pixel rounded half away
 *     from zero;
 *   - output: the native-scale disparity in 1/256 pixel,
 *     floor(((256 xl - (256 (xr + s*) + offset)) S_l + 2^15) / 2^16) with
 *     S_l = round(65536 * 1.2^l), and the least SAD; INT32_MIN and
 *     0xFFFFFFFF when not refined.
 */
#include <stdint.h>
#include <stdlib.h>

#include "oracle.h"

static int32_t level_pixel(const uint8_t *pyr, int32_t W, int32_t H, int32_t l, int32_t x, int32_t y) {
    int64_t at = 0;
    for (int32_t k = 0; k < l; k++) {
        int32_t w, h;
        or_level_size(W, H, k, &w, &h);
        at += (int64_t)w * h;
    }
    int32_t w, h;
    or_level_size(W, H, l, &w, &h);
    return pyr[at + (int64_t)y * w + x];
}

void or_stereo_refine(const uint8_t *pyr_l, const uint8_t *pyr_r, int32_t W, int32_t H, int32_t nl,
                      const or_kps *L, const or_kps *R, const int32_t *idx, int32_t w, int32_t r,
                      int32_t *disp_q8, uint32_t *sad_min) {
    int64_t *sad = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * r + 1));
    for (int32_t i = 0; i < nl; i++) {
        disp_q8[i] = INT32_MIN;
        sad_min[i] = 0xFFFFFFFFu;
        int32_t j = idx[i];
        if (j < 0) continue;
        int32_t l = L->level[i];
        int32_t wl, hl;
        or_level_size(W, H, l, &wl, &hl);
        int32_t xl = L->x[i], yl = L->y[i], xr = R->x[j];
        if (xl - w < 0 || xl + w >= wl || yl - w < 0 || yl + w >= hl) continue;
        if (xr - r - w < 0 || xr + r + w >= wl) continue;
        for (int32_t s = -r; s <= r; s++) {
            int64_t acc = 0;
            for (int32_t dy = -w; dy <= w; dy++)
                for (int32_t dx = -w; dx <= w; dx++) {
                    int32_t a = level_pixel(pyr_l, W, H, l, xl + dx, yl + dy);
                    int32_t b = level_pixel(pyr_r, W, H, l, xr + s + dx, yl + dy);
                    acc += a > b ? a - b : b - a;
                }
            sad[s + r] = acc;
        }
        int32_t best = 0;
        for (int32_t s = -r; s <= r; s++) {
            int64_t v = sad[s + r], bv = sad[best + r];
            int32_t as = s < 0 ? -s : s, ab = best < 0 ? -best : best;
            if (v < bv || (v == bv && (as < ab || (as == ab && s < best)))) best = s;
        }
        if (best == -r || best == r) continue;
        int64_t sm = sad[best - 1 + r], s0 = sad[best + r], sp = sad[best + 1 + r];
        int64_t den = sm - 2 * s0 + sp;
        int64_t off = 0;
        if (den != 0) {
            int64_t num = 128 * (sm - sp);                 /* offset = num / den, in 1/256 pixel */
            int64_t mag = num < 0 ? -num : num;
            int64_t q = (2 * mag + den) / (2 * den);       /* round half away from zero */
            off = num < 0 ? -q : q;
        }
        int64_t d_level = 256 * (int64_t)xl - (256 * (int64_t)(xr + best) + off);
        int64_t num0 = d_level * or_scale_q16(l) + 32768;
        /* floor division by 2^16 (also for a negative disparity) */
        int64_t d0 = num0 >= 0 ? num0 / 65536 : -((-num0 + 65535) / 65536);
        disp_q8[i] = (int32_t)d0;
        sad_min[i] = (uint32_t)s0;
    }
    free(sad);
}
