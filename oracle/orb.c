/*
 * Oracle: Gaussian smoothing, ORB orientation and rBRIEF (test
 * infrastructure only).
 *
 * Sec. III-2 smooths every level with a Gaussian before extracting ORB
 * descriptors for all scales at once.  The paper names ORB but fixes no
 * constants; the readings adopted here:
 *   Smoothing: separable 7-tap kernel [18 33 49 56 49 33 18] / 256
 *     (a sigma = 2 Gaussian quantised to sum 256), horizontal pass then
 *     vertical pass, clamp-to-edge, each pass rounded (sum + 128) >> 8.
 *   Orientation: intensity centroid of the unsmoothed level over the disc
 *     u^2 + v^2 <= 225, m10 = sum u I, m01 = sum v I; the direction is
 *     quantised to the nearest multiple of 12 degrees (30 bins) by exact
 *     integer comparison against the bin boundaries at 6 + 12 j degrees,
 *     stored in Q14.  m = (0, 0) gives bin 0.
 *   rBRIEF: 256 pairs (p, q) in the disc (an input), rotated by bin k with
 *     the Q14 table (C_k, S_k) and rounded half away from zero; bit i is
 *     [B(x + p_i') < B(x + q_i')] on the smoothed level; bit i is word
 *     i >> 5, bit i & 31.
 */
#include <math.h>
#include <stdlib.h>
#include "oracle.h"

static const int32_t TAPS[7] = {18, 33, 49, 56, 49, 33, 18};

static int32_t clampi(int32_t v, int32_t lo, int32_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

void or_blur_level(const uint8_t *lvl, int32_t W, int32_t H, uint8_t *out) {
    uint8_t *tmp = (uint8_t *)malloc((size_t)W * H);
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int32_t s = 0;
            for (int32_t k = -3; k <= 3; k++) s += TAPS[k + 3] * lvl[(int64_t)y * W + clampi(x + k, 0, W - 1)];
            tmp[(int64_t)y * W + x] = (uint8_t)((s + 128) >> 8);
        }
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int32_t s = 0;
            for (int32_t k = -3; k <= 3; k++) s += TAPS[k + 3] * tmp[(int64_t)clampi(y + k, 0, H - 1) * W + x];
            out[(int64_t)y * W + x] = (uint8_t)((s + 128) >> 8);
        }
    free(tmp);
}

void or_rot_table(int32_t *C, int32_t *S) {
    for (int32_t k = 0; k < 30; k++) {
        double a = (double)k * 12.0 * M_PI / 180.0;
        C[k] = (int32_t)lround(16384.0 * cos(a));
        S[k] = (int32_t)lround(16384.0 * sin(a));
    }
}

void or_bin_table(int32_t *bx, int32_t *by) {
    for (int32_t j = 0; j < 30; j++) {
        double a = (6.0 + 12.0 * (double)j) * M_PI / 180.0;
        bx[j] = (int32_t)lround(16384.0 * cos(a));
        by[j] = (int32_t)lround(16384.0 * sin(a));
    }
}

void or_moments(const uint8_t *lvl, int32_t pitch, int32_t x, int32_t y,
                int64_t *m10, int64_t *m01) {
    int64_t a = 0, b = 0;
    for (int32_t v = -15; v <= 15; v++)
        for (int32_t u = -15; u <= 15; u++) {
            if (u * u + v * v > 225) continue;
            int32_t I = lvl[(int64_t)(y + v) * pitch + (x + u)];
            a += (int64_t)u * I;
            b += (int64_t)v * I;
        }
    *m10 = a;
    *m01 = b;
}

/* upper half-plane (angles in [0, 180)) -> 0, lower -> 1 */
static int half(int64_t x, int64_t y) { return (y < 0 || (y == 0 && x < 0)) ? 1 : 0; }

/* angle(a) >= angle(b), angles measured in [0, 360) */
static int angle_ge(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
    int ha = half(ax, ay), hb = half(bx, by);
    if (ha != hb) return ha > hb;
    return bx * ay - by * ax >= 0;
}

int32_t or_angle_bin(int64_t mx, int64_t my) {
    if (mx == 0 && my == 0) return 0;
    int32_t bx[30], by[30], cnt = 0;
    or_bin_table(bx, by);
    for (int32_t j = 0; j < 30; j++)
        if (angle_ge(mx, my, bx[j], by[j])) cnt++;
    return cnt % 30;
}

static int32_t rhaz(int64_t a) {
    int64_t m = a < 0 ? -a : a;
    int64_t r = (m + 8192) >> 14;
    return (int32_t)(a < 0 ? -r : r);
}

static void rotate(const int32_t *C, const int32_t *S, int32_t u, int32_t v, int32_t k,
                   int32_t *ur, int32_t *vr) {
    *ur = rhaz((int64_t)u * C[k] - (int64_t)v * S[k]);
    *vr = rhaz((int64_t)u * S[k] + (int64_t)v * C[k]);
}

void or_rotate_point(int32_t u, int32_t v, int32_t k, int32_t *ur, int32_t *vr) {
    int32_t C[30], S[30];
    or_rot_table(C, S);
    rotate(C, S, u, v, k, ur, vr);
}

void or_describe(const uint8_t *pyr, int32_t W, int32_t H, const or_params *p,
                 const int8_t *pattern, int32_t n, or_kps *kps) {
    if (p->border < 15 || p->n_levels > 16) return;   /* the disc must stay inside the level */
    /* per-level views and smoothed copies */
    const uint8_t *lv[16];
    uint8_t *bl[16];
    int32_t lw[16], lh[16];
    const uint8_t *at = pyr;
    int32_t C[30], S[30];
    or_rot_table(C, S);
    for (int32_t l = 0; l < p->n_levels; l++) {
        or_level_size(W, H, l, &lw[l], &lh[l]);
        lv[l] = at;
        bl[l] = (uint8_t *)malloc((size_t)lw[l] * lh[l]);
        if (p->blur)
            or_blur_level(at, lw[l], lh[l], bl[l]);
        else
            for (int64_t q = 0; q < (int64_t)lw[l] * lh[l]; q++) bl[l][q] = at[q];
        at += (int64_t)lw[l] * lh[l];
    }
    for (int32_t i = 0; i < n; i++) {
        int32_t l = kps->level[i], x = kps->x[i], y = kps->y[i];
        int64_t m10, m01;
        or_moments(lv[l], lw[l], x, y, &m10, &m01);
        int32_t k = or_angle_bin(m10, m01);
        kps->bin[i] = (uint8_t)k;
        if (!kps->desc) continue;
        uint32_t *d = kps->desc + 8 * (int64_t)i;
        for (int32_t w = 0; w < 8; w++) d[w] = 0;
        for (int32_t t = 0; t < 256; t++) {
            int32_t pu, pv, qu, qv;
            rotate(C, S, pattern[4 * t + 0], pattern[4 * t + 1], k, &pu, &pv);
            rotate(C, S, pattern[4 * t + 2], pattern[4 * t + 3], k, &qu, &qv);
            int32_t a = bl[l][(int64_t)(y + pv) * lw[l] + (x + pu)];
            int32_t b = bl[l][(int64_t)(y + qv) * lw[l] + (x + qu)];
            if (a < b) d[t >> 5] |= 1u << (t & 31);
        }
    }
    for (int32_t l = 0; l < p->n_levels; l++) free(bl[l]);
}
