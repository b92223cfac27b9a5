/*
 * Oracle: multiscale detection = FAST/BR + Feature Culling per level,
 * Pyramidal Feature Aggregation and the keypoint cap (test infrastructure).
 *
 * PFA follows the three steps of Sec. II-C-2:
 *   1. every culled keypoint of level n is projected to the native scale,
 *      x0 = x_n * 1.2^n (rounded with the Q16 factor S_n, see pyramid.c),
 *      and its response is written into a zero-initialised
 *      M[N_s][H][W];
 *   2. K_r = sum over levels of M, K_l = number of levels with M > 0;
 *   3. a sparse q x q NMS (q = 2 r + 1, r = 1 by default) runs only around
 *      keypoints: a keypoint is suppressed when some other position of its
 *      window holds a better (K_l, K_r) pair.  The text says "smaller k_r
 *      and k_l"; the default reading is a lexicographic comparison of
 *      (K_l, K_r) (mode 0), the literal "both strictly smaller" reading is
 *      mode 1.  Positions with equal pairs do not suppress each other.
 *   Survivors keep every per-level member (Fig. "pfa").
 * Cap: when more than n_max keypoints survive, the first n_max by
 *   (K_l desc, K_r desc, level asc, cell_y asc, cell_x asc) are kept; output
 *   stays in canonical order (level, cell_y, cell_x).
 * Learned gating: with a level-0 cell mask, a level-l cell is evaluated only
 *   if its footprint at the native scale, [x S_l >> 16, ceil((x + c_l) S_l / 2^16)),
 *   overlaps a kept level-0 cell (same in y); other cells are empty.
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static int better(int32_t kl_h, int32_t kr_h, int32_t kl_g, int32_t kr_g, int32_t mode) {
    if (mode == 0) return kl_h > kl_g || (kl_h == kl_g && kr_h > kr_g);
    return kl_h > kl_g && kr_h > kr_g;
}

int32_t or_pfa_from_records(int32_t n, const int32_t *level, const int32_t *x0,
                            const int32_t *y0, const int32_t *resp, int32_t W, int32_t H,
                            int32_t n_levels, int32_t nms_mode, int32_t nms_radius,
                            int32_t *kl, int32_t *kr, int32_t *keep) {
    int64_t plane = (int64_t)W * H;
    int32_t *M = (int32_t *)calloc((size_t)(plane * n_levels), sizeof(int32_t));
    int32_t *Kr = (int32_t *)calloc((size_t)plane, sizeof(int32_t));
    int32_t *Kl = (int32_t *)calloc((size_t)plane, sizeof(int32_t));
    int32_t rc = 0;
    if (!M || !Kr || !Kl) { rc = -1; goto done; }
    /* step 1: projection into M */
    for (int32_t i = 0; i < n; i++) {
        int64_t at = (int64_t)level[i] * plane + (int64_t)y0[i] * W + x0[i];
        if (M[at] != 0) { rc = -2; goto done; }   /* two keypoints of one level on one pixel */
        M[at] = resp[i];
    }
    /* step 2: K_r and K_l */
    for (int32_t l = 0; l < n_levels; l++)
        for (int64_t q = 0; q < plane; q++) {
            int32_t m = M[(int64_t)l * plane + q];
            Kr[q] += m;
            Kl[q] += m > 0;
        }
    /* step 3: sparse NMS around each keypoint */
    for (int32_t i = 0; i < n; i++) {
        int64_t g = (int64_t)y0[i] * W + x0[i];
        kl[i] = Kl[g];
        kr[i] = Kr[g];
        int32_t sup = 0;
        for (int32_t dy = -nms_radius; dy <= nms_radius; dy++)
            for (int32_t dx = -nms_radius; dx <= nms_radius; dx++) {
                int32_t xx = x0[i] + dx, yy = y0[i] + dy;
                if ((dx == 0 && dy == 0) || xx < 0 || yy < 0 || xx >= W || yy >= H) continue;
                int64_t h = (int64_t)yy * W + xx;
                if (Kl[h] > 0 && better(Kl[h], Kr[h], Kl[g], Kr[g], nms_mode)) sup = 1;
            }
        keep[i] = !sup;
    }
done:
    free(M);
    free(Kr);
    free(Kl);
    return rc;
}

typedef struct {
    int32_t kl, kr, idx;
} rank_t;

static int rank_cmp(const void *a, const void *b) {
    const rank_t *p = (const rank_t *)a, *q = (const rank_t *)b;
    if (p->kl != q->kl) return p->kl > q->kl ? -1 : 1;
    if (p->kr != q->kr) return p->kr > q->kr ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

int32_t or_cell_runs(int32_t l, int32_t cx, int32_t cy, int32_t c, int32_t W0, int32_t H0,
                     int32_t cell0, const uint8_t *mask0) {
    if (!mask0) return 1;
    int64_t S = or_scale_q16(l);
    int32_t ncx0 = (W0 + cell0 - 1) / cell0, ncy0 = (H0 + cell0 - 1) / cell0;
    int64_t fx0 = ((int64_t)cx * c * S) >> 16;
    int64_t fx1 = ((int64_t)(cx * c + c) * S + 65535) >> 16;
    int64_t fy0 = ((int64_t)cy * c * S) >> 16;
    int64_t fy1 = ((int64_t)(cy * c + c) * S + 65535) >> 16;
    int64_t a0 = fx0 / cell0, a1 = (fx1 - 1) / cell0, b0 = fy0 / cell0, b1 = (fy1 - 1) / cell0;
    if (a1 > ncx0 - 1) a1 = ncx0 - 1;
    if (b1 > ncy0 - 1) b1 = ncy0 - 1;
    for (int64_t b = b0; b <= b1; b++)
        for (int64_t a = a0; a <= a1; a++)
            if (mask0[b * ncx0 + a]) return 1;
    return 0;
}

int32_t or_detect(const uint8_t *pyr, int32_t W, int32_t H, const or_params *p,
                  const uint8_t *cell_mask0, or_kps *out) {
    if (p->n_levels < 1 || p->n_levels > 16 || p->border < 3 || p->p_min > p->p_max ||
        p->cell0 < 1 || p->cell0 > 32 || p->n_max < 1 || p->eps_lo > p->eps_hi)
        return -1;
    /* culled records of all levels in canonical order */
    int32_t cap = 0;
    for (int32_t l = 0; l < p->n_levels; l++) {
        int32_t w, h, c = or_cell_size(p->cell0, l);
        or_level_size(W, H, l, &w, &h);
        if (c < 1) return -1;
        cap += ((w + c - 1) / c) * ((h + c - 1) / c);
    }
    int32_t *R_level = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *R_x = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *R_y = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *R_x0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *R_y0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *R_s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *R_f = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *R_kl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *R_kr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int32_t *R_keep = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    rank_t *rk = (rank_t *)malloc(sizeof(rank_t) * (size_t)(cap + 1));
    int32_t n = 0, rc = 0;
    const uint8_t *lvl = pyr;
    for (int32_t l = 0; l < p->n_levels; l++) {
        int32_t w, h, c = or_cell_size(p->cell0, l);
        or_level_size(W, H, l, &w, &h);
        int32_t ncx = (w + c - 1) / c, ncy = (h + c - 1) / c;
        uint32_t *key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)ncx * ncy);
        uint8_t *flag = (uint8_t *)malloc((size_t)ncx * ncy);
        or_cull_level(lvl, w, h, c, p, key, flag);
        for (int32_t cy = 0; cy < ncy; cy++)
            for (int32_t cx = 0; cx < ncx; cx++) {
                uint32_t k = key[cy * ncx + cx];
                if (!k || !or_cell_runs(l, cx, cy, c, W, H, p->cell0, cell_mask0)) continue;
                int32_t idx = 1023 - (int32_t)(k & 1023u);
                R_level[n] = l;
                R_x[n] = cx * c + idx % c;
                R_y[n] = cy * c + idx / c;
                R_x0[n] = or_project(R_x[n], l, W);
                R_y0[n] = or_project(R_y[n], l, H);
                R_s[n] = (int32_t)(k >> 10);
                R_f[n] = flag[cy * ncx + cx];
                n++;
            }
        free(key);
        free(flag);
        lvl += (int64_t)w * h;
    }
    if (p->pfa) {
        rc = or_pfa_from_records(n, R_level, R_x0, R_y0, R_s, W, H, p->n_levels, p->nms_mode,
                                 p->nms_radius, R_kl, R_kr, R_keep);
        if (rc) { rc = -1; goto done; }
    } else {
        for (int32_t i = 0; i < n; i++) {
            R_kl[i] = 1;
            R_kr[i] = R_s[i];
            R_keep[i] = 1;
        }
    }
    /* cap */
    int32_t m = 0;
    for (int32_t i = 0; i < n; i++)
        if (R_keep[i]) {
            rk[m].kl = R_kl[i];
            rk[m].kr = R_kr[i];
            rk[m].idx = i;
            m++;
        }
    if (m > p->n_max) {
        qsort(rk, (size_t)m, sizeof(rank_t), rank_cmp);
        for (int32_t i = 0; i < n; i++) R_keep[i] = 0;
        for (int32_t j = 0; j < p->n_max; j++) R_keep[rk[j].idx] = 1;
        m = p->n_max;
    }
    if (m > out->capacity) { rc = -1; goto done; }
    int32_t o = 0;
    for (int32_t i = 0; i < n; i++) {
        if (!R_keep[i]) continue;
        out->x[o] = (uint16_t)R_x[i];
        out->y[o] = (uint16_t)R_y[i];
        out->level[o] = (uint8_t)R_level[i];
        out->flags[o] = (uint8_t)R_f[i];
        out->score[o] = (uint16_t)R_s[i];
        out->x0[o] = (uint16_t)R_x0[i];
        out->y0[o] = (uint16_t)R_y0[i];
        out->kl[o] = (uint8_t)R_kl[i];
        out->kr[o] = (uint32_t)R_kr[i];
        out->bin[o] = 0;
        o++;
    }
    rc = o;
done:
    free(R_level); free(R_x); free(R_y); free(R_x0); free(R_y0); free(R_s); free(R_f);
    free(R_kl); free(R_kr); free(R_keep); free(rk);
    return rc;
}
