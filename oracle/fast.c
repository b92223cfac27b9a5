/*
 * Oracle: FAST labelling with Bounded Rectification, corner response and
 * Feature Culling (test infrastructure only).
 *
 * Ring: the 16 pixels of the radius-3 Bresenham circle in cyclic order, as
 * drawn in the paper's non-corner figure (Sec. II-A).
 * Labels (Eq. 1): bright if I_p > I_c + eps, dark if I_p < I_c - eps, else
 *   similar.  Eq. 1 leaves |I_p - I_c| = eps unlabelled; it is read as
 *   similar.
 * Counts: N_b / N_d = the longest cyclic run of contiguous bright / dark
 *   ring pixels (16 when the whole ring has the label).
 * Corner (Eq. 3, Bounded Rectification): P_min <= N_b <= P_max or
 *   P_min <= N_d <= P_max.  Eq. 2/3 write "N_b, N_d"; both at once is
 *   impossible for P_min > 8, so it is read as "either".  P_max = 16 gives
 *   plain FAST (Eq. 2).
 * Response (Sec. III-1): sum over the 16 ring pixels of |I_c - I_p|.
 * Feature Culling (Sec. II-C-1): non-overlapping c x c cells tiled from the
 *   level origin (last row/column may be partial); the strongest response
 *   in a cell survives.  Ties go to the first pixel in raster order within
 *   the cell: key = (score << 10) | (1023 - ((y - y_cell) c + (x - x_cell))).
 *   With a fallback threshold eps_lo >= 0, a cell with no corner at eps_hi
 *   takes its strongest eps_lo corner and is flagged.
 */
#include "oracle.h"

static const int32_t RING_DX[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
static const int32_t RING_DY[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

int32_t or_longest_run(const int32_t lab[16]) {
    int32_t all = 1;
    for (int32_t k = 0; k < 16; k++)
        if (!lab[k]) all = 0;
    if (all) return 16;
    int32_t best = 0;
    for (int32_t s = 0; s < 16; s++) {
        int32_t n = 0;
        while (n < 16 && lab[(s + n) % 16]) n++;
        if (n > best) best = n;
    }
    return best;
}

int32_t or_mask_is_corner(uint32_t mask16, int32_t p_min, int32_t p_max) {
    int32_t lab[16];
    for (int32_t k = 0; k < 16; k++) lab[k] = (int32_t)((mask16 >> k) & 1u);
    int32_t n = or_longest_run(lab);
    return p_min <= n && n <= p_max;
}

int32_t or_is_corner(const uint8_t *lvl, int32_t pitch, int32_t x, int32_t y,
                     int32_t eps, int32_t p_min, int32_t p_max, int32_t *nb, int32_t *nd) {
    int32_t c = lvl[(int64_t)y * pitch + x];
    int32_t b[16], d[16];
    for (int32_t k = 0; k < 16; k++) {
        int32_t p = lvl[(int64_t)(y + RING_DY[k]) * pitch + (x + RING_DX[k])];
        b[k] = p > c + eps;
        d[k] = p < c - eps;
    }
    int32_t n_b = or_longest_run(b), n_d = or_longest_run(d);
    if (nb) *nb = n_b;
    if (nd) *nd = n_d;
    return (p_min <= n_b && n_b <= p_max) || (p_min <= n_d && n_d <= p_max);
}

int32_t or_score(const uint8_t *lvl, int32_t pitch, int32_t x, int32_t y) {
    int32_t c = lvl[(int64_t)y * pitch + x], s = 0;
    for (int32_t k = 0; k < 16; k++) {
        int32_t p = lvl[(int64_t)(y + RING_DY[k]) * pitch + (x + RING_DX[k])];
        s += p > c ? p - c : c - p;
    }
    return s;
}

/* Corner response matrix: score at corners, 0 elsewhere and in the border. */
void or_crf(const uint8_t *lvl, int32_t W, int32_t H, int32_t eps, int32_t p_min,
            int32_t p_max, int32_t border, uint16_t *crf) {
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            uint16_t v = 0;
            if (x >= border && x < W - border && y >= border && y < H - border &&
                or_is_corner(lvl, W, x, y, eps, p_min, p_max, 0, 0))
                v = (uint16_t)or_score(lvl, W, x, y);
            crf[(int64_t)y * W + x] = v;
        }
}

void or_cull_level(const uint8_t *lvl, int32_t W, int32_t H, int32_t c,
                   const or_params *p, uint32_t *key, uint8_t *flag) {
    int32_t ncx = (W + c - 1) / c, ncy = (H + c - 1) / c;
    for (int32_t cy = 0; cy < ncy; cy++)
        for (int32_t cx = 0; cx < ncx; cx++) {
            uint32_t best_hi = 0, best_lo = 0;
            for (int32_t y = cy * c; y < (cy + 1) * c && y < H; y++)
                for (int32_t x = cx * c; x < (cx + 1) * c && x < W; x++) {
                    if (x < p->border || x >= W - p->border || y < p->border || y >= H - p->border)
                        continue;
                    uint32_t idx = (uint32_t)((y - cy * c) * c + (x - cx * c));
                    uint32_t s = (uint32_t)or_score(lvl, W, x, y);
                    uint32_t k = (s << 10) | (1023u - idx);
                    if (or_is_corner(lvl, W, x, y, p->eps_hi, p->p_min, p->p_max, 0, 0) && k > best_hi)
                        best_hi = k;
                    if (p->eps_lo >= 0 &&
                        or_is_corner(lvl, W, x, y, p->eps_lo, p->p_min, p->p_max, 0, 0) && k > best_lo)
                        best_lo = k;
                }
            int64_t ci = (int64_t)cy * ncx + cx;
            if (best_hi) {
                key[ci] = best_hi;
                flag[ci] = 0;
            } else if (best_lo) {
                key[ci] = best_lo;
                flag[ci] = 1;
            } else {
                key[ci] = 0;
                flag[ci] = 0;
            }
        }
}
