/*
 * Oracle: image pyramid at scale factor 1.2 (test infrastructure only).
 *
 * The paper builds a multiscale pyramid with scale factor 1.2 on the GPU
 * (Sec. III-2; the 1.2 factor is stated in the PyCA cell-size ablation of
 * Sec. IV-F).  It does not say how levels are resampled.  Reading adopted:
 *   - level sizes  W_l = floor(W / 1.2^l + 1/2), evaluated in exact integers
 *     as floor((2 W 5^l + 6^l) / (2 * 6^l));
 *   - level l is resampled from level l-1 (chained), bilinear with a
 *     half-pixel-centre mapping whose source coordinate is floored to Q8;
 *   - the four 8-bit weights give a Q16 sum rounded half-up.
 */
#include "oracle.h"

static int64_t ipow(int64_t b, int32_t e) {
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

void or_level_size(int32_t W, int32_t H, int32_t l, int32_t *Wl, int32_t *Hl) {
    int64_t n = ipow(5, l), d = ipow(6, l);
    *Wl = (int32_t)((2 * (int64_t)W * n + d) / (2 * d));
    *Hl = (int32_t)((2 * (int64_t)H * n + d) / (2 * d));
}

/* Cell side at level l: floor(cell0 * 5^l / 6^l), so that 32-pixel cells
 * become 8-pixel cells at the eighth level, as Sec. IV-F states. */
int32_t or_cell_size(int32_t cell0, int32_t l) {
    return (int32_t)(((int64_t)cell0 * ipow(5, l)) / ipow(6, l));
}

/* S_l = round(65536 * 1.2^l) = round(65536 * 6^l / 5^l). */
int64_t or_scale_q16(int32_t l) {
    int64_t n = 65536 * ipow(6, l), d = ipow(5, l);
    return (2 * n + d) / (2 * d);
}

/* Projection of a level-l coordinate to the native scale, x0 = x * 1.2^l
 * (Sec. II-C-2), rounded to nearest with S_l in Q16 and clamped to the image. */
int32_t or_project(int32_t x, int32_t l, int32_t W0) {
    int64_t v = ((int64_t)x * or_scale_q16(l) + 32768) >> 16;
    if (v > W0 - 1) v = W0 - 1;
    return (int32_t)v;
}

int64_t or_pyramid_bytes(int32_t W, int32_t H, int32_t L) {
    int64_t s = 0;
    for (int32_t l = 0; l < L; l++) {
        int32_t w, h;
        or_level_size(W, H, l, &w, &h);
        s += (int64_t)w * h;
    }
    return s;
}

/* One output coordinate of the chained resize: Q8 source position. */
static void src_coord(int32_t o, int32_t n_src, int32_t n_dst, int32_t *a, int32_t *b, int32_t *f) {
    int64_t t = (((int64_t)(2 * o + 1)) * n_src - n_dst) * 128 / n_dst;
    *a = (int32_t)(t >> 8);
    *f = (int32_t)(t & 255);
    *b = (*a + 1 < n_src) ? *a + 1 : n_src - 1;
}

void or_pyramid(const uint8_t *img, int32_t W, int32_t H, int32_t pitch,
                int32_t L, uint8_t *out) {
    /* level 0 is the input */
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++)
            out[(int64_t)y * W + x] = img[(int64_t)y * pitch + x];
    uint8_t *prev = out;
    int32_t pw = W, ph = H;
    for (int32_t l = 1; l < L; l++) {
        int32_t w, h;
        or_level_size(W, H, l, &w, &h);
        uint8_t *cur = prev + (int64_t)pw * ph;
        for (int32_t y = 0; y < h; y++) {
            int32_t ya, yb, fy;
            src_coord(y, ph, h, &ya, &yb, &fy);
            for (int32_t x = 0; x < w; x++) {
                int32_t xa, xb, fx;
                src_coord(x, pw, w, &xa, &xb, &fx);
                int32_t p_aa = prev[(int64_t)ya * pw + xa];
                int32_t p_ab = prev[(int64_t)ya * pw + xb];
                int32_t p_ba = prev[(int64_t)yb * pw + xa];
                int32_t p_bb = prev[(int64_t)yb * pw + xb];
                int32_t v = (256 - fx) * (256 - fy) * p_aa + fx * (256 - fy) * p_ab
                          + (256 - fx) * fy * p_ba + fx * fy * p_bb;
                cur[(int64_t)y * w + x] = (uint8_t)((v + 32768) >> 16);
            }
        }
        prev = cur;
        pw = w;
        ph = h;
    }
}
