/*
 * CPU oracle of the stereo front-end (test infrastructure only).
 *
 * A plain, slow, scalar C implementation of what the front-end computes,
 * written from the paper's definitions: FAST labelling and Bounded
 * Rectification (Sec. II-A, Eq. 1-3), the corner response of Sec. III-1,
 * Feature Culling (Sec. II-C-1), Pyramidal Feature Aggregation
 * (Sec. II-C-2, Fig. "pfa"), Gaussian smoothing + ORB orientation and
 * rBRIEF (Sec. III-2) and descriptor-distance stereo matching (Sec. III-3).
 * Choices the paper leaves open are fixed as documented at each function.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or constant
 * generator with the GPU library.
 */
#ifndef FRONTEND_ORACLE_H
#define FRONTEND_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t eps_hi, eps_lo, p_min, p_max, border, n_levels, cell0;
    int32_t pfa, nms_mode, nms_radius, n_max, blur, d_max, match_th, row_band;
} or_params;

/* Level geometry. */
void    or_level_size(int32_t W, int32_t H, int32_t l, int32_t *Wl, int32_t *Hl);
int32_t or_cell_size(int32_t cell0, int32_t l);
int64_t or_scale_q16(int32_t l);
int32_t or_project(int32_t x, int32_t l, int32_t W0);

/* Pyramid: levels 0..L-1 packed back to back, each with pitch W_l. */
int64_t or_pyramid_bytes(int32_t W, int32_t H, int32_t L);
void    or_pyramid(const uint8_t *img, int32_t W, int32_t H, int32_t pitch,
                   int32_t L, uint8_t *out);

/* FAST + Bounded Rectification on one level. */
int32_t or_longest_run(const int32_t lab[16]);
int32_t or_is_corner(const uint8_t *lvl, int32_t pitch, int32_t x, int32_t y,
                     int32_t eps, int32_t p_min, int32_t p_max, int32_t *nb, int32_t *nd);
int32_t or_score(const uint8_t *lvl, int32_t pitch, int32_t x, int32_t y);
void    or_crf(const uint8_t *lvl, int32_t W, int32_t H, int32_t eps, int32_t p_min,
               int32_t p_max, int32_t border, uint16_t *crf);
int32_t or_mask_is_corner(uint32_t mask16, int32_t p_min, int32_t p_max);

/* Feature Culling on one level: key and fallback flag per cell (row-major). */
void    or_cull_level(const uint8_t *lvl, int32_t W, int32_t H, int32_t c,
                      const or_params *p, uint32_t *key, uint8_t *flag);

/* Output keypoints of one image (SoA, canonical order level, cell_y, cell_x). */
typedef struct {
    uint16_t *x, *y;
    uint8_t  *level, *flags;
    uint16_t *score, *x0, *y0;
    uint8_t  *kl;
    uint32_t *kr;
    uint8_t  *bin;
    uint32_t *desc;       /* 8 words per keypoint, may be NULL */
    int32_t   capacity;
} or_kps;

/* Detection: pyramid + FAST/BR + FC + PFA + cap.  Returns the keypoint count,
 * or -1 on invalid parameters / insufficient capacity. */
int32_t or_detect(const uint8_t *pyr, int32_t W, int32_t H, const or_params *p,
                  const uint8_t *cell_mask0, or_kps *out);

/* Learned gating: does level-l cell (cx, cy) of side c run under the level-0
 * cell mask (ncx0 x ncy0 bytes, row-major)?  1 when mask0 is NULL. */
int32_t or_cell_runs(int32_t l, int32_t cx, int32_t cy, int32_t c, int32_t W0, int32_t H0,
                     int32_t cell0, const uint8_t *mask0);

/* PFA from a given per-cell key list (used by the figure replay as well). */
int32_t or_pfa_from_records(int32_t n, const int32_t *level, const int32_t *x0,
                            const int32_t *y0, const int32_t *resp, int32_t W, int32_t H,
                            int32_t n_levels, int32_t nms_mode, int32_t nms_radius,
                            int32_t *kl, int32_t *kr, int32_t *keep);

/* Smoothing, orientation, descriptor. */
void    or_blur_level(const uint8_t *lvl, int32_t W, int32_t H, uint8_t *out);
void    or_rot_table(int32_t *C, int32_t *S);
void    or_bin_table(int32_t *bx, int32_t *by);
void    or_moments(const uint8_t *lvl, int32_t pitch, int32_t x, int32_t y,
                   int64_t *m10, int64_t *m01);
int32_t or_angle_bin(int64_t mx, int64_t my);
void    or_rotate_point(int32_t u, int32_t v, int32_t k, int32_t *ur, int32_t *vr);
void    or_describe(const uint8_t *pyr, int32_t W, int32_t H, const or_params *p,
                    const int8_t *pattern, int32_t n, or_kps *kps);

/* Stereo matching of one pair (left, right keypoints with descriptors). */
void    or_stereo(int32_t nl, const or_kps *L, int32_t nr, const or_kps *R,
                  const or_params *p, int32_t *idx, uint16_t *dist, int16_t *disp);

/* Sub-pixel refinement of the stereo matches of one pair by SAD
 * minimisation on the keypoints' levels (packed pyramids of both views);
 * disp_q8: native-scale disparity in 1/256 pixel (INT32_MIN if not
 * refined), sad_min: the least SAD (0xFFFFFFFF if not refined). */
void    or_stereo_refine(const uint8_t *pyr_l, const uint8_t *pyr_r, int32_t W, int32_t H, int32_t nl,
                         const or_kps *L, const or_kps *R, const int32_t *idx, int32_t w, int32_t r,
                         int32_t *disp_q8, uint32_t *sad_min);

/* Descriptor matching of query keypoints against reference keypoints:
 * candidates within `radius` native pixels (x and y) and `level_band`
 * levels; least Hamming distance (ties: smaller index), runner-up distance;
 * accepted if best <= match_th and (ratio_pct > 0 with a runner-up)
 * 100 best < ratio_pct second.  idx -1 if not accepted; dist1 / dist2
 * 0xFFFF when absent. */
void    or_feature_match(int32_t nq, const or_kps *Q, int32_t nr, const or_kps *R, int32_t radius,
                         int32_t level_band, int32_t match_th, int32_t ratio_pct, int32_t *idx,
                         uint16_t *dist1, uint16_t *dist2);

/* Whole front-end for one stereo pair; returns 0 on success. */
int32_t or_frontend_pair(const uint8_t *left, const uint8_t *right, int32_t W, int32_t H,
                         const or_params *p, const int8_t *pattern,
                         or_kps *kl, int32_t *nl, or_kps *kr, int32_t *nr,
                         int32_t *idx, uint16_t *dist, int16_t *disp);

#ifdef __cplusplus
}
#endif
#endif
