/*
 * Oracle: the whole front-end for one rectified stereo pair (test
 * infrastructure only): pyramid, detection, description of both views, then
 * stereo matching of the left keypoints against the right ones.
 */
#include <stdlib.h>
#include "oracle.h"

int32_t or_frontend_pair(const uint8_t *left, const uint8_t *right, int32_t W, int32_t H,
                         const or_params *p, const int8_t *pattern,
                         or_kps *kl, int32_t *nl, or_kps *kr, int32_t *nr,
                         int32_t *idx, uint16_t *dist, int16_t *disp) {
    int64_t bytes = or_pyramid_bytes(W, H, p->n_levels);
    uint8_t *pl = (uint8_t *)malloc((size_t)bytes), *pr = (uint8_t *)malloc((size_t)bytes);
    int32_t rc = 0;
    or_pyramid(left, W, H, W, p->n_levels, pl);
    or_pyramid(right, W, H, W, p->n_levels, pr);
    *nl = or_detect(pl, W, H, p, 0, kl);
    *nr = or_detect(pr, W, H, p, 0, kr);
    if (*nl < 0 || *nr < 0) {
        rc = -1;
    } else {
        or_describe(pl, W, H, p, pattern, *nl, kl);
        or_describe(pr, W, H, p, pattern, *nr, kr);
        or_stereo(*nl, kl, *nr, kr, p, idx, dist, disp);
    }
    free(pl);
    free(pr);
    return rc;
}
