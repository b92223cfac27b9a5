/*
 * Oracle: descriptor matching of a frame's keypoints against reference
 * keypoints (the previous frame's, or map points projected into the frame):
 * the middle-end's "Descriptor Matching" beside "Conic Projections" (Sec.
 * III-3, Fig. "slampipeline"), test infrastructure only.
 *
 * The paper names the step without its rules; the reading taken here:
 *   - reference j is a candidate of query i when their native-scale
 *     positions differ by at most `radius` in x and in y (a square window
 *     around the query, whose reference positions are the predicted ones)
 *     and their pyramid levels by at most `level_band`;
 *   - distance = Hamming distance of the 256-bit descriptors;
 *   - best = the candidate of least distance, ties to the smaller index;
 *     second = the least distance among the other candidates;
 *   - accepted when best <= match_th and, with ratio_pct > 0 and a second
 *     candidate, 100 * best < ratio_pct * second (the nearest-neighbour
 *     ratio test);
 *   - outputs per query: the reference index (-1 if not accepted), the best
 *     and second distances (0xFFFF when absent), whatever the acceptance.
 */
#include "oracle.h"

static int32_t hamming256(const uint32_t *a, const uint32_t *b) {
    int32_t c = 0;
    for (int32_t w = 0; w < 8; w++) {
        uint32_t v = a[w] ^ b[w];
        while (v) {
            c += (int32_t)(v & 1u);
            v >>= 1;
        }
    }
    return c;
}

void or_feature_match(int32_t nq, const or_kps *Q, int32_t nr, const or_kps *R, int32_t radius,
                      int32_t level_band, int32_t match_th, int32_t ratio_pct, int32_t *idx, uint16_t *dist1,
                      uint16_t *dist2) {
    for (int32_t i = 0; i < nq; i++) {
        int32_t best = -1, bd = 0, sd = -1;
        for (int32_t j = 0; j < nr; j++) {
            int32_t dx = (int32_t)Q->x0[i] - (int32_t)R->x0[j];
            int32_t dy = (int32_t)Q->y0[i] - (int32_t)R->y0[j];
            int32_t dl = (int32_t)Q->level[i] - (int32_t)R->level[j];
            if (dx < -radius || dx > radius || dy < -radius || dy > radius) continue;
            if (dl < -level_band || dl > level_band) continue;
            int32_t h = hamming256(Q->desc + 8 * (int64_t)i, R->desc + 8 * (int64_t)j);
            if (best < 0 || h < bd) {
                if (best >= 0) sd = bd;        /* the former best becomes the runner-up */
                best = j;
                bd = h;
            } else if (sd < 0 || h < sd) {
                sd = h;                        /* j > best here: ties keep the smaller index */
            }
        }
        dist1[i] = best >= 0 ? (uint16_t)bd : 0xFFFF;
        dist2[i] = sd >= 0 ? (uint16_t)sd : 0xFFFF;
        int32_t ok = best >= 0 && bd <= match_th;
        if (ok && ratio_pct > 0 && sd >= 0) ok = 100 * bd < ratio_pct * sd;
        idx[i] = ok ? best : -1;
    }
}
