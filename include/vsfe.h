/*
 * vsfe.h - C ABI of the MI355X (gfx950) stereo visual-SLAM front-end.
 *
 * The library computes, for a batch of images (stereo pairs are images 2i
 * and 2i+1), the GPU front-end of "High-Speed Stereo Visual SLAM for
 * Low-Powered Computing Devices" (Kumar, Park, Behera, RA-L 2023):
 *   pyramid_build        image pyramid at scale 1.2 (Sec. III-2)
 *   fast_br_detect       FAST with Bounded Rectification (Sec. II-A, Eq. 1-3),
 *                        corner response (Sec. III-1), fused Feature Culling
 *                        (Sec. II-C-1)
 *   pyca_cull_aggregate  Pyramidal Feature Aggregation with sparse NMS
 *                        (Sec. II-C-2, Fig. "pfa") and the keypoint cap
 *   orb_describe         smoothing, ORB orientation, rBRIEF (Sec. III-2)
 *   stereo_match         descriptor-distance stereo matching along
 *                        rectified rows (Sec. III-3, middle-end)
 *   stereo_refine        sub-pixel refinement of the matches by correlation
 *                        (SAD) minimisation (Sec. III-3, middle-end)
 *   feature_match        descriptor matching against the previous frame or
 *                        projected map points (Sec. III-3, middle-end)
 *   fc_cull_crf          Feature Culling over a materialised response matrix
 *                        with the paper's thread schemes (ablation)
 *   cnn_*                learned cell proposer gating the detector
 *
 * Conventions (all calls):
 *   - Return value: VSFE_OK or a negative VSFE_E* code.  On error nothing is
 *     launched and vsfe_last_error() describes the cause.
 *   - Hot-path calls are asynchronous on the caller's HIP stream (passed as
 *     void*, NULL = the default stream).  They never allocate, never
 *     synchronise and never abort; they launch kernels only, so they can be
 *     captured into a HIP graph.
 *   - All buffers are device memory owned by the caller, sized with
 *     vsfe_batch_info_get().  The library owns only the context (constant
 *     tables) and the batch object (its device work tables); both are made
 *     at set-up time.
 *   - A context and a batch are used from one stream at a time.
 *   - `status` is a caller-zeroed device int32; kernels OR VSFE_DEV_* bits
 *     into it for conditions only the device can see.
 */
#ifndef VSFE_H
#define VSFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VSFE_OK            0
#define VSFE_EINVAL       -1   /* null pointer, bad size or parameter      */
#define VSFE_ECAPACITY    -2   /* a size limit of the library is exceeded  */
#define VSFE_EHIP         -3   /* a HIP call failed (see vsfe_last_error)  */
#define VSFE_EUNSUPPORTED -4   /* no gfx950 device / feature not built     */

#define VSFE_DEV_OVERFLOW  1   /* a device-side count exceeded capacity    */

#define VSFE_MAX_LEVELS   12
#define VSFE_MAX_IMAGES   4096
#define VSFE_MAX_DIM      8192
#define VSFE_KP_FALLBACK  1u   /* kp flags bit: found at the fallback threshold */
#define VSFE_KEY_FALLBACK (1u << 22)   /* cell-key bit: fallback threshold  */

/*
 * Front-end parameters.  Defaults (vsfe_params_default) follow the paper:
 * eps = 20 (Sec. II-A), P_min = 9, P_max = 13 (Eq. 3), 32x32 cells at the
 * native scale, q = 3 NMS window (Sec. II-C-2), 8 levels at scale 1.2.
 */
typedef struct vsfe_params {
    int32_t eps_hi;      /* FAST threshold, 0..254                              */
    int32_t eps_lo;      /* per-cell fallback threshold, -1 = none, <= eps_hi    */
    int32_t p_min;       /* shortest accepted contiguous run, 1..16              */
    int32_t p_max;       /* longest accepted run (16 = plain FAST), >= p_min     */
    int32_t border;      /* skipped pixels at each level edge, >= 3 (>= 15 to describe) */
    int32_t n_levels;    /* pyramid levels, 1..VSFE_MAX_LEVELS                   */
    int32_t cell0;       /* native-scale cell side, 8..32; level l uses
                            floor(cell0 * 5^l / 6^l), which must stay >= 1       */
    int32_t pfa;         /* 1 = pyramidal feature aggregation, 0 = culling only  */
    int32_t nms_mode;    /* 0 = (k_l, k_r) lexicographic, 1 = both larger         */
    int32_t nms_radius;  /* NMS half-window at the native scale, 0..3 (q = 2r+1) */
    int32_t n_max;       /* keypoints kept per image, 1..65535                   */
    int32_t blur;        /* 1 = 7-tap smoothing before rBRIEF sampling           */
    int32_t d_max;       /* stereo disparity range at the native scale, >= 0     */
    int32_t match_th;    /* largest accepted Hamming distance, 0..256            */
    int32_t row_band;    /* |dy| tolerance in level pixels, 0..3                 */
} vsfe_params;

/* Keypoints, structure of arrays.  Image i owns slots
 * [i * n_max, i * n_max + kp_count[i]) in canonical order (level, cell row,
 * cell column).  x, y are level coordinates, x0, y0 their projection to
 * the native scale; kl / kr are the aggregated level count / response sum
 * of the keypoint's native-scale position; bin is the orientation in 12-
 * degree steps (written by orb_describe). */
typedef struct vsfe_kp_soa {
    uint16_t *x, *y;
    uint8_t  *level, *flags;
    uint16_t *score, *x0, *y0;
    uint8_t  *kl;
    uint32_t *kr;
    uint8_t  *bin;
} vsfe_kp_soa;

typedef struct vsfe_batch_info {
    int64_t input_bytes;      /* smallest input buffer covering every image    */
    int64_t pyr_bytes;        /* pyramid buffer (levels 1..n_levels-1)         */
    int64_t crf_elems;        /* uint16 elements of the optional response dump */
    int64_t n_cells;          /* cell_keys elements (all images, all levels)   */
    int64_t n_cells0;         /* level-0 cells (cell_mask / cell_logits size)  */
    int64_t kp_capacity;      /* keypoint slots = n_images * n_max             */
    int64_t workspace_bytes;  /* pyca_cull_aggregate workspace                 */
    int64_t match_capacity;   /* stereo outputs = n_pairs * n_max              */
    int32_t n_images;
    int32_t n_levels;
    int32_t n_det_items;      /* detector work items (256-thread blocks) with the
                                 batch's current tiles                          */
    int32_t reserved;
} vsfe_batch_info;

typedef struct vsfe_level_info {
    int32_t width, height, pitch;   /* level size and row pitch in bytes      */
    int32_t cell, ncx, ncy;         /* cell side and cell grid                */
    int64_t offset;                 /* level 0: byte offset in the input
                                       buffer; others: in the pyramid buffer */
    int64_t cell_offset;            /* first cell of this level in cell_keys  */
    int64_t crf_offset;             /* first element in the response dump     */
    int64_t cell0_offset;           /* first level-0 cell of the image        */
} vsfe_level_info;

typedef struct vsfe_ctx vsfe_ctx;
typedef struct vsfe_batch vsfe_batch;

/* ---------------------------------------------------------------- set-up */

/* Fill *p with the paper's defaults (see vsfe_params).  Host only. */
void vsfe_params_default(vsfe_params *p);

/* Validate parameters without touching the GPU.  Host only. */
int32_t vsfe_params_check(const vsfe_params *p);

/* Level geometry of a W x H image (Sec. III-2 pyramid, Sec. IV-F cell
 * shrink): W_l = floor(W / 1.2^l + 1/2), cell_l = floor(cell0 * 5^l / 6^l).
 * Host only; EINVAL for bad sizes. */
int32_t vsfe_level_geometry(const vsfe_params *p, int32_t W, int32_t H, int32_t level,
                            int32_t *Wl, int32_t *Hl, int32_t *cell);

/* Create a context on the current HIP device.  `pattern` is a host array of
 * 256 x 4 int8 (pu, pv, qu, qv) test-point pairs inside the radius-15 disc;
 * the library stores the 30 rotated copies.  Synchronous.  Errors: EINVAL
 * (bad params / pattern outside the disc), EUNSUPPORTED (no gfx950),
 * EHIP. */
int32_t vsfe_ctx_create(const vsfe_params *p, const int8_t *pattern, vsfe_ctx **out);
int32_t vsfe_ctx_destroy(vsfe_ctx *ctx);

/* Describe a batch of n images.  widths/heights/pitches/offsets are host
 * arrays of n entries; image i occupies bytes offsets[i] .. offsets[i] +
 * pitches[i] * heights[i] of the caller's input buffer.  Builds and uploads
 * the device work tables (synchronous, set-up time).  Errors: EINVAL
 * (sizes, a level with no cell, pitch < width), ECAPACITY (n > VSFE_MAX_IMAGES). */
int32_t vsfe_batch_create(const vsfe_ctx *ctx, int32_t n, const int32_t *widths,
                          const int32_t *heights, const int32_t *pitches,
                          const int64_t *offsets, vsfe_batch **out);
int32_t vsfe_batch_destroy(vsfe_batch *b);

/* Buffer sizes of a batch without creating it (host only, same arguments
 * and errors as vsfe_batch_create). */
int32_t vsfe_batch_plan(const vsfe_params *p, int32_t n, const int32_t *widths,
                        const int32_t *heights, const int32_t *pitches,
                        const int64_t *offsets, vsfe_batch_info *out);
int32_t vsfe_batch_info_get(const vsfe_batch *b, vsfe_batch_info *out);
int32_t vsfe_batch_level_info(const vsfe_batch *b, int32_t image, int32_t level,
                              vsfe_level_info *out);

/* Tile shape of fast_br_detect: the target tile extent in pixels (each
 * level packs as many whole cells as fit, at least one).  Host only; takes
 * effect for batches created afterwards.  EINVAL unless 8 <= tw <= 128,
 * 8 <= th <= 32. */
int32_t vsfe_ctx_set_tile(vsfe_ctx *ctx, int32_t tile_w, int32_t tile_h);

/* ------------------------------------------------------- batch autotuner */

/* Outcome of vsfe_batch_autotune, per pyramid level l < n_levels. */
typedef struct {
    int32_t n_levels;
    int32_t tile_w[VSFE_MAX_LEVELS];   /* chosen detector tile, pixels (whole cells) */
    int32_t tile_h[VSFE_MAX_LEVELS];
    float us[VSFE_MAX_LEVELS];         /* mean launch time of the chosen shape, microseconds */
    float us_before[VSFE_MAX_LEVELS];  /* ... of the shape the batch had before tuning */
    int32_t n_tried[VSFE_MAX_LEVELS];  /* distinct shapes timed */
    float us_worst[VSFE_MAX_LEVELS];   /* slowest shape timed (the landscape's spread) */
    float us_median[VSFE_MAX_LEVELS];  /* median over the shapes timed */
    int32_t pyr_schedule;              /* chosen pyramid schedule (VSFE_PYR_LEVELS / _TOWER) */
    int32_t pyr_tile_w, pyr_tile_h;    /* ... and single-launch tile */
    float pyr_us;                      /* pyramid_build time of the chosen schedule, microseconds */
    float pyr_us_before;               /* ... of the schedule the batch had before tuning */
    float pyr_us_worst;                /* slowest schedule timed */
    int32_t pyr_n_tried;               /* schedules timed (0 with one level) */
} vsfe_tune_report;

/* Per-level detector tile extents of a batch (host arrays of n_levels
 * entries).  A tile of tw x th pixels at level l packs
 * min(32, max(1, tw / cell_l)) x min(4, max(1, th / cell_l)) cells.
 * Results never depend on the tiles.  set: EINVAL unless every level has
 * 8 <= tw <= 128 and 8 <= th <= 32; synchronises the device and replaces
 * the batch's detector work table, so HIP graphs captured earlier with this
 * batch must be captured again. */
int32_t vsfe_batch_tiles_get(const vsfe_batch *b, int32_t *tile_w, int32_t *tile_h);
int32_t vsfe_batch_set_tiles(vsfe_batch *b, const int32_t *tile_w, const int32_t *tile_h);

/* Pyramid schedule of a batch (results never depend on it):
 *   VSFE_PYR_LEVELS  one launch per level, each level from the previous one
 *                    in HBM;
 *   VSFE_PYR_TOWER   one launch for all levels: a block stages a level-0
 *                    window and builds its tile of every level in LDS, with
 *                    the halo the smaller levels need (tile_w x tile_h is
 *                    the owned tile at level 1);
 *   VSFE_PYR_AUTO    (default) TOWER for batches of at most 2^26 level-0
 *                    pixels where its plan fits, else LEVELS (measured:
 *                    TOWER wins on small and mixed batches, where levels are
 *                    launch- and latency-bound; LEVELS on 64 1080p pairs,
 *                    where it streams HBM).
 * tile_w / tile_h: 0 = default (112 x 32, or 64 x 16 when the batch has
 * fewer than 512 blocks of 112 x 32); else 16..240 columns, a multiple
 * of 4, and 4..64 rows.  Host only; a new tile synchronises the device and
 * replaces the batch's plan tables, so HIP graphs captured earlier with this
 * batch must be captured again.  Errors: EINVAL (unknown schedule, tile out
 * of range), ECAPACITY (TOWER requested but its block does not fit; a tile
 * that does not fit leaves the default tile planned), EHIP.
 * pyramid_build_levels always uses one launch per level. */
#define VSFE_PYR_AUTO   0
#define VSFE_PYR_LEVELS 1
#define VSFE_PYR_TOWER  2
int32_t vsfe_batch_set_pyramid(vsfe_batch *b, int32_t schedule, int32_t tile_w, int32_t tile_h);
/* The schedule pyramid_build will use (LEVELS or TOWER) and the planned
 * single-launch tile. */
int32_t vsfe_batch_pyramid_get(const vsfe_batch *b, int32_t *schedule, int32_t *tile_w, int32_t *tile_h);

/* Batching autotuner.  First times pyramid_build under the batch's current
 * schedule, one launch per level and single-launch tiles from 48 x 8 to
 * 240 x 32 (those whose block fits), and installs the fastest as by
 * vsfe_batch_set_pyramid; `pyr` is rewritten with the same bytes.  Then,
 * for every pyramid level, times fast_br_detect (no cell mask) over that
 * level of every image of the batch for each distinct whole-cell tile shape
 * that fits the detector's 128 x 32 pixel block (one warm-up and `reps`
 * timed launches each, HIP events on `stream`), keeps the fastest per level
 * and installs it as by vsfe_batch_set_tiles.  `images` and `pyr` must hold
 * the batch's data with the pyramid built; `cell_keys` (n_cells entries) is
 * overwritten.  Set-up call: synchronous, allocates a
 * temporary table, not capturable.  Errors: EINVAL (null pointers, reps
 * outside 1..1000), EHIP. */
int32_t vsfe_batch_autotune(const vsfe_ctx *ctx, vsfe_batch *b, const uint8_t *images,
                            const uint8_t *pyr, uint32_t *cell_keys, int32_t *status,
                            int32_t reps, void *stream, vsfe_tune_report *out);

/* ---------------------------------------------- measurement aids (not the
 * paper's method): device ceilings the kernels are compared against. */

/* kind VSFE_PROBE_VALU: `blocks` x 256 threads, each running 8 independent
 * float FMA chains for 128 x iters VALU instructions per wave (plus a few);
 * kind VSFE_PROBE_LDS: each thread reads 16 x iters conflict-free 16-byte
 * LDS words (ds_read_b128, 1 KB per wave instruction).  sink: device
 * buffer of blocks x 256 x 4 bytes (written only in a case that does not
 * occur, so that the work is kept); clocks (device, 2 x uint64, written):
 * shader-clock cycles and 100 MHz wall-clock ticks that block 0 spent in
 * its loop, whose ratio is the clock the device ran at.  Time the call with
 * events on `stream`.  Errors: EINVAL (kind, blocks or iters outside
 * 1..2^20, blocks x iters above 2^26, null buffers), EHIP. */
#define VSFE_PROBE_VALU 1
#define VSFE_PROBE_LDS  2
int32_t vsfe_probe(int32_t kind, int32_t blocks, int32_t iters, void *sink, uint64_t *clocks, void *stream);

/* Last error message of the calling thread ("" if none). */
const char *vsfe_last_error(void);

/* --------------------------------------------------------------- hot path */

/* Sec. III-2: levels 1..n-1 of every image, each resampled from the level
 * above by bilinear interpolation at half-pixel centres with Q8 source
 * coordinates (floored) and Q16 weights rounded half up.  images: input
 * buffer (level 0, read), pyr: pyramid buffer (written). */
int32_t pyramid_build(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                      uint8_t *pyr, int32_t *status, void *stream);

/* pyramid_build restricted to levels level_begin <= l < level_end
 * (1 <= level_begin): each from level l - 1, which must already be built.
 * Lets later levels be built on a second stream while an earlier level is
 * consumed (the learned proposer needs levels 1..3 only).  Errors: EINVAL
 * (null buffers, an empty or out-of-range level range), EHIP. */
int32_t pyramid_build_levels(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images, uint8_t *pyr,
                             int32_t level_begin, int32_t level_end, int32_t *status, void *stream);

/* Sec. II-A Eq. 1-3, Sec. III-1 and Sec. II-C-1: for every pixel inside the
 * border of every level, FAST labels at eps_hi (and eps_lo), the longest
 * cyclic bright / dark run N, the Bounded-Rectification test
 * p_min <= N <= p_max, the response sum |I_c - I_p| over the 16-pixel ring,
 * and per cell the maximum key (score << 10) | (1023 - offset in cell),
 * falling back to eps_lo corners (bit VSFE_KEY_FALLBACK) when the cell has
 * no eps_hi corner.  cell_keys (n_cells, written, 0 = empty).
 * cell_mask (n_cells0 bytes, nullable): learned gating, a level-l cell runs
 * only if its native-scale footprint overlaps a non-zero level-0 cell; the
 * keys of other cells are 0.  The gated launch visits only the tiles with a
 * running cell (a device-built work list; the others cost one early exit).
 * crf_debug (crf_elems, nullable): per-pixel eps_hi response, 0 elsewhere
 * (and 0 in cells that a cell_mask skips). */
int32_t fast_br_detect(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                       const uint8_t *pyr, const uint8_t *cell_mask, uint32_t *cell_keys,
                       uint16_t *crf_debug, int32_t *status, void *stream);

/* fast_br_detect restricted to levels level_begin <= l < level_end (same
 * results for those levels' cells, other cells untouched), without the
 * response dump.  Level 0 reads only the input, so its detection can run on
 * a second stream while pyramid_build writes the other levels; calls with
 * disjoint level ranges write disjoint cells and may run concurrently.
 * pyr may be null when the range is level 0 only.  Errors: EINVAL (null
 * pointers, an empty or out-of-range level range), EHIP. */
int32_t fast_br_detect_levels(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                              const uint8_t *pyr, const uint8_t *cell_mask, uint32_t *cell_keys,
                              int32_t level_begin, int32_t level_end, int32_t *status, void *stream);

/* Sec. II-C-2 (PFA): projection of every culled keypoint to the native
 * scale (x0 = round(x * 1.2^l) in Q16), K_l / K_r per native position,
 * sparse (2r+1)^2 NMS around keypoints, survivors kept at every level, then
 * the cap to n_max by (k_l desc, k_r desc, canonical order).  With
 * params.pfa = 0: culling output only (k_l = 1, k_r = score) and the cap.
 * Writes kps (kp_capacity slots) and kp_count (n_images).  workspace:
 * workspace_bytes of device scratch. */
int32_t pyca_cull_aggregate(const vsfe_ctx *ctx, const vsfe_batch *b,
                            const uint32_t *cell_keys, void *workspace,
                            const vsfe_kp_soa *kps, int32_t *kp_count, int32_t *status,
                            void *stream);

/* pyca_cull_aggregate for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same results, with the per-cell scratch taken from a fixed device
 * array of the library (VSFE_NOALLOC_MAX_CELLS uint32 = 16 MiB per GPU,
 * held until the process ends; its address is resolved at context
 * creation) instead of a workspace argument.  Allocates nothing.  Every
 * call on one GPU shares that array and leaves its contents behind (each
 * call writes every rank it reads, nothing needs clearing): calls that
 * overlap on one GPU, from any stream or context, race.  Errors: as
 * pyca_cull_aggregate, plus ECAPACITY when the batch has more than
 * VSFE_NOALLOC_MAX_CELLS cells. */
#define VSFE_NOALLOC_MAX_CELLS (1 << 22)
int32_t pyca_cull_aggregate_noalloc(const vsfe_ctx *ctx, const vsfe_batch *b, const uint32_t *cell_keys,
                                    const vsfe_kp_soa *kps, int32_t *kp_count, int32_t *status, void *stream);

/* Sec. III-2: intensity-centroid orientation over the radius-15 disc of the
 * unsmoothed level, quantised to 30 bins; 256 binary tests on the
 * bin-rotated pattern over the smoothed level.  Writes kps.bin and desc
 * (8 uint32 per keypoint slot; bit t is word t >> 5, bit t & 31).
 * Requires params.border >= 15 (EINVAL otherwise). */
int32_t orb_describe(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                     const uint8_t *pyr, const vsfe_kp_soa *kps, const int32_t *kp_count,
                     uint32_t *desc, int32_t *status, void *stream);

/* Sec. III-3: for each left keypoint (image 2i) the right keypoint (image
 * 2i+1) of the same level with |dy| <= row_band and native-scale disparity
 * d = x0_l - x0_r in [0, d_max] of least Hamming distance (ties: smaller
 * |dy|, smaller d, smaller index); accepted if distance <= match_th.
 * Outputs (match_capacity, slot pair * n_max + i): match_idx (right index
 * or -1), match_dist (0xFFFF if none), match_disp (-1 if none).  The
 * keypoints must be in canonical order, as pyca_cull_aggregate writes them
 * (in any other order the matches are unspecified, and every read stays
 * inside the image's slots).  EINVAL if the batch has an odd image count or
 * a pair of unequal sizes. */
int32_t stereo_match(const vsfe_ctx *ctx, const vsfe_batch *b, const vsfe_kp_soa *kps,
                     const int32_t *kp_count, const uint32_t *desc, int32_t *match_idx,
                     uint16_t *match_dist, int16_t *match_disp, int32_t *status, void *stream);

/* Sec. III-3 (the middle-end's stereo matcher pairs correlation
 * minimisation with descriptor-distance minimisation): sub-pixel refinement
 * of the stereo matches.  For each left keypoint slot i < kp_count of pair p
 * with match_idx[p * n_max + i] = j >= 0 (as written by stereo_match): on
 * the keypoint's level of both views (unsmoothed), SAD(s) of the
 * (2 half_window + 1)^2 window around the left keypoint against the window
 * around the right keypoint's column shifted by s in [-search_radius,
 * search_radius], same rows; s* = least SAD (ties: smaller |s|, then smaller
 * s); the vertex of the parabola through SAD(s* - 1), SAD(s*), SAD(s* + 1),
 * offset (S- - S+) / (2 (S- - 2 S0 + S+)) in 1/256 pixel rounded half away
 * from zero (0 if the denominator is 0).  Outputs (match_capacity entries,
 * same slots as stereo_match; entries of slots >= kp_count untouched):
 * disp_q8 = native-scale disparity in 1/256 pixel,
 * floor(((256 x_l - (256 (x_r + s*) + offset)) S_l + 2^15) / 2^16),
 * INT32_MIN when not refined (no match, a window leaving the level, or
 * s* = +-search_radius); sad_min (nullable) = SAD(s*), 0xFFFFFFFF when not
 * refined.  EINVAL: half_window or search_radius outside 1..7, an odd image
 * count or a pair of unequal sizes, null buffers. */
int32_t stereo_refine(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images, const uint8_t *pyr,
                      const vsfe_kp_soa *kps, const int32_t *kp_count, const int32_t *match_idx,
                      int32_t half_window, int32_t search_radius, int32_t *disp_q8, uint32_t *sad_min,
                      int32_t *status, void *stream);

/* Sec. III-3 (the middle-end's "Descriptor Matching" beside "Conic
 * Projections", Fig. "slampipeline"): match the keypoints of a frame (the
 * query: image i's slots [i n_max, i n_max + query_count[i]) of `query`,
 * descriptors query_desc) against reference keypoints laid out the same way
 * (the previous frame's results, or map points whose x0 / y0 hold their
 * predicted native-scale positions and level their predicted level).  A
 * reference is a candidate when |x0_q - x0_r| <= radius, |y0_q - y0_r| <=
 * radius (native pixels) and |level_q - level_r| <= level_band; best = least
 * Hamming distance (ties: smaller reference index), second = least distance
 * among the other candidates; accepted when best <= match_th and, with
 * ratio_pct > 0 and a second candidate, 100 best < ratio_pct second.
 * Outputs per query slot (kp_capacity entries): match_idx (reference index
 * within the image, -1 if not accepted), dist1 / dist2 (0xFFFF if absent).
 * workspace: vsfe_feature_match_workspace() bytes of 16-byte aligned
 * device scratch (overwritten; it holds the references bucketed by cell with
 * copies of their descriptors).  EINVAL: radius outside 0..255, level_band
 * outside 0..11, match_th outside 0..256, ratio_pct outside 0..100, null
 * buffers, a misaligned workspace. */
int32_t vsfe_feature_match_workspace(const vsfe_batch *b, int64_t *bytes);
int32_t feature_match(const vsfe_ctx *ctx, const vsfe_batch *b, const vsfe_kp_soa *query,
                      const int32_t *query_count, const uint32_t *query_desc, const vsfe_kp_soa *ref,
                      const int32_t *ref_count, const uint32_t *ref_desc, int32_t radius, int32_t level_band,
                      int32_t match_th, int32_t ratio_pct, void *workspace, int32_t *match_idx, uint16_t *dist1,
                      uint16_t *dist2, int32_t *status, void *stream);

/* Sec. II-C-1 as the paper schedules it, kept as an ablation beside the
 * fused culling of fast_br_detect: Feature Culling over a materialised
 * response matrix `crf` (the crf_debug output of fast_br_detect) of one
 * pyramid level of every image, with square cells of side `cell` (1..32):
 * per cell the largest key (response << 10) | (1023 - offset in cell),
 * 0 = no corner (the keys of fast_br_detect without a fallback threshold).
 * scheme 0: multi-location-per-thread culling (ceil(cell / n_loc) threads
 * per column, n_loc rows each, then the column maxima at a stride) with
 * thread-efficient warp allocation (128-thread-wide blocks packing
 * floor(128 / cell) cells); scheme 1: log2 tree reduction, one block and
 * one thread per pixel of a cell; scheme 2: scheme 0 with one block per
 * cell.  keys: image i's cells row-major from i * stride
 * (vsfe_fc_cull_stride), keys_elems = its size in entries, at least
 * n_images x stride for this level and cell (ECAPACITY otherwise, before
 * any launch).  EINVAL: level out of range, cell outside 1..32, scheme
 * outside 0..2, n_loc outside 1..32 or ceil(cell / n_loc) > 8 (schemes 0
 * and 2). */
int32_t vsfe_fc_cull_stride(const vsfe_batch *b, int32_t level, int32_t cell, int64_t *stride);
int32_t fc_cull_crf(const vsfe_ctx *ctx, const vsfe_batch *b, const uint16_t *crf, int32_t level, int32_t cell,
                    int32_t scheme, int32_t n_loc, uint32_t *keys, int64_t keys_elems, int32_t *status,
                    void *stream);

/* ---------------------------------------------------- learned cell proposer
 *
 * Not part of the paper: a small CNN on pyramid level 3 predicts which
 * native-scale cells will hold final keypoints; fast_br_detect's cell_mask
 * then skips the others.  Network: x = (I_3 - 128) / 128, three 3x3
 * stride-2 convolutions with zero padding 1 (1 -> 16 -> 32 -> 32 channels,
 * ReLU) and a 1x1 head (32 -> 1), one logit per stride-8 grid position.
 * Parameters: one vector of 14081 values, OIHW weights then biases per
 * layer (w1 b1 w2 b2 w3 b3 w4 b4); the kernels read a bfloat16 copy, so
 * the network evaluated is the bfloat16-valued one, with float32 sums.
 * cnn_forward (training) feeds each convolution its float32 input as a
 * bfloat16 value + remainder pair (logits within about 1e-4 of float32);
 * cnn_propose (inference) stores activations as float16 (within 1e-2 of
 * float32; weights beyond +-65504 saturate there).  Grid logits are float32,
 * images' grids back to back in image order, row-major.  All calls need
 * n_levels >= 4 (EINVAL otherwise) and a workspace of workspace_bytes. */
typedef struct vsfe_cnn_info {
    int64_t workspace_bytes;  /* activations, gradients, partial sums        */
    int64_t grid_elems;       /* grid logits of all images                   */
    int64_t n_cells0;         /* native-scale cells (cell_mask size)         */
    int32_t n_params;         /* 14081                                       */
} vsfe_cnn_info;

int32_t vsfe_cnn_info_get(const vsfe_batch *b, vsfe_cnn_info *out);

/* Forward pass on level 3 of every image (pyr = pyramid buffer after
 * pyramid_build); writes grid_logits and keeps activations in the
 * workspace for cnn_backward. */
int32_t cnn_forward(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *pyr,
                    const uint16_t *params_bf16, void *workspace, float *grid_logits,
                    int32_t *status, void *stream);

/* Forward pass, then per native-scale cell the maximum logit of the grid
 * positions whose projected centre ((8 j + 4) S_3 + 2^15) >> 16 lies in the
 * cell (+inf if none).  cell_mask[c] = logit >= thresh (cells without a
 * position are kept).  cell_logits is nullable. */
int32_t cnn_propose(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *pyr,
                    const uint16_t *params_bf16, float thresh, void *workspace,
                    float *grid_logits, float *cell_logits, uint8_t *cell_mask,
                    int32_t *status, void *stream);

/* Gradient of the mean binary cross-entropy over all grid positions,
 * positives weighted by pos_weight (> 0), w.r.t. the parameters; needs the
 * workspace of a cnn_forward with the same parameters and inputs.  grad:
 * 14081 float32 (overwritten); loss: one float32 (nullable).
 * Deterministic (fixed-order reductions). */
int32_t cnn_backward(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *pyr,
                     const uint16_t *params_bf16, void *workspace, const float *grid_logits,
                     const float *grid_targets, float pos_weight, float *grad, float *loss,
                     int32_t *status, void *stream);

/* One Adam step (bias-corrected, step >= 1) on n float32 parameters; also
 * refreshes their bfloat16 copy (round to nearest even). */
int32_t cnn_adam_step(float *params, uint16_t *params_bf16, float *m, float *v,
                      const float *grad, int32_t n, float lr, float beta1, float beta2,
                      float eps, int32_t step, void *stream);

#ifdef __cplusplus
}
#endif
#endif
