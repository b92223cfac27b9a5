/*
 * Oracle: rectified-row stereo matching by descriptor-distance minimisation
 * (Sec. III-3, the middle-end's stereo matcher), test infrastructure only.
 *
 * For left keypoint i the candidates are right keypoints j of the same
 * pyramid level whose level row differs by at most row_band and whose
 * native-scale disparity d = x0_i - x0_j lies in [0, d_max].  The match is
 * the candidate of least Hamming distance over the 256-bit descriptors;
 * ties go to the smaller |dy|, then the smaller d, then the smaller j.  It
 * is accepted when the distance is at most match_th; otherwise
 * idx = -1, dist = 0xFFFF, disp = -1.
 */
#include "oracle.h"

static int32_t popcount32(uint32_t v) {
    int32_t c = 0;
    while (v) {
        c += (int32_t)(v & 1u);
        v >>= 1;
    }
    return c;
}

void or_stereo(int32_t nl, const or_kps *L, int32_t nr, const or_kps *R,
               const or_params *p, int32_t *idx, uint16_t *dist, int16_t *disp) {
    for (int32_t i = 0; i < nl; i++) {
        int32_t best = -1, bd = 0, bdy = 0, bdisp = 0;
        for (int32_t j = 0; j < nr; j++) {
            if (R->level[j] != L->level[i]) continue;
            int32_t dy = (int32_t)L->y[i] - (int32_t)R->y[j];
            if (dy < 0) dy = -dy;
            if (dy > p->row_band) continue;
            int32_t d = (int32_t)L->x0[i] - (int32_t)R->x0[j];
            if (d < 0 || d > p->d_max) continue;
            int32_t h = 0;
            for (int32_t w = 0; w < 8; w++) h += popcount32(L->desc[8 * (int64_t)i + w] ^ R->desc[8 * (int64_t)j + w]);
            int take = best < 0 || h < bd || (h == bd && (dy < bdy || (dy == bdy && d < bdisp)));
            if (take) {
                best = j;
                bd = h;
                bdy = dy;
                bdisp = d;
            }
        }
        if (best >= 0 && bd <= p->match_th) {
            idx[i] = best;
            dist[i] = (uint16_t)bd;
            disp[i] = (int16_t)bdisp;
        } else {
            idx[i] = -1;
            dist[i] = 0xFFFF;
            disp[i] = -1;
        }
    }
}
