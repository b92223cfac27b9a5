// Internal declarations of the gfx950 front-end library (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "vsfe.h"

namespace vsfe {

// Per-level geometry as the kernels see it (one 64-byte record).
struct LevelDev {
    int32_t w, h, pitch, cell;
    int32_t ncx, ncy, scale_q16;
    int32_t xtab, ytab;    // first entries of the resampling tables (levels >= 1)
    int32_t row_tab;       // row-start table entry of this level's cell row 0
    int64_t offset;        // level 0: into the input buffer, else into the pyramid buffer
    int64_t cell_offset;   // global index of the first cell of this level
    int64_t crf_offset;    // first element of this level in the response dump
};
static_assert(sizeof(LevelDev) == 64, "LevelDev layout");

struct ImageDev {
    int32_t w, h, n_levels, row_tab_end;   // row_tab_end: the image's last row-start entry
    int64_t cell_base;     // first cell of the image (level 0)
    int64_t n_cells;       // cells over all levels
    int64_t cell0_offset;  // first level-0 cell in mask / logit arrays
    int64_t kp_offset;     // first keypoint slot
    LevelDev lv[VSFE_MAX_LEVELS];
};

// Output tile of the pyramid kernel: PYR_TW x PYR_TH pixels of one level,
// resampled from a staged source window of at most PYR_SH x PYR_SW bytes
// starting at (xs, ys) of the level above (xs and ncols are multiples of 16).
constexpr int PYR_TW = 256;   // 64 lanes x 4 columns
constexpr int PYR_TH = 32;    // 4 waves x 8 rows
constexpr int PYR_SW = 336;
constexpr int PYR_SH = 44;
// One output tile of one level with both levels' geometry copied in (32-bit
// fields: the block reads its item with scalar loads, no dependent load of
// the level records).
struct PyrItem {
    int64_t src_offset, dst_offset;           // level l-1 / level l in their buffers
    int32_t sw, sh, spitch, dw, dh, dpitch;   // source and output level sizes and pitches
    int32_t xtab, ytab;                       // output level's resampling table entries
    int32_t tx, ty, xs, ys, ncols, nrows;     // tile, staged source window
};
static_assert(sizeof(PyrItem) == 72, "PyrItem layout");

// Single-launch pyramid ("tower"): a block owns one tile of every level of
// one image (the tiles of level l partition it; those of level l+1 are the
// outputs whose source falls in the block's tile of level l) and computes,
// in LDS, the range of each level that its own tile and the next level's
// computed range need.  Column and row plans are separate (the resampling
// is separable); a block pairs one of each.
constexpr int TWR_TW = 112;    // default owned tile at level 1, columns (multiple of 4)
constexpr int TWR_TH = 32;     // ... rows
constexpr int TWR_STAGE = 4;   // level-0 window: at most 4 x 256 16-byte chunks
constexpr int TWR_TAB = 2048;  // table entries in LDS (both plans, all levels)
constexpr int TWR_LDS = 60 * 1024;   // dynamic LDS limit (tables + two level buffers)
constexpr int64_t TWR_AUTO_PIXELS = (int64_t)1 << 26;   // default schedule: single launch up to this many level-0 pixels
constexpr int TWR_SMALL_ITEMS = 512;   // fewer blocks than this at the default tile: plan 64 x 16 instead
// One plan of one axis (columns: quad-aligned ranges, level 0 16-aligned).
struct TowerAxis {
    int16_t c0[VSFE_MAX_LEVELS], cn[VSFE_MAX_LEVELS];  // computed range (level 0: staged window)
    int16_t o0[VSFE_MAX_LEVELS], o1[VSFE_MAX_LEVELS];  // owned range [o0, o1), levels >= 1
};
static_assert(sizeof(TowerAxis) == 96, "TowerAxis layout");
struct TowerItem {
    int64_t src_offset;                 // level 0 of the image in the input buffer
    int32_t sw, sh, spitch;             // its size and pitch
    int32_t xs, ys, ncols, nrows;       // staged level-0 window (xs, ncols multiples of 16)
    int32_t image, ax, ay;              // image record, column plan, row plan
    int32_t tabx, ntabx, taby, ntaby;   // table entries of the two plans (levels 1.. in order)
    int32_t odd_off;                    // LDS offset of the odd levels' buffer (even ones at 0)
    int32_t pad;
};
static_assert(sizeof(TowerItem) == 72, "TowerItem layout");

// Detector block: DET_WAVES waves of 64 lanes; a tile is at most 128 pixels
// wide and 8 rows per wave high, at most 32 x DET_WAVES cells.
#ifndef VSFE_DET_WAVES
#define VSFE_DET_WAVES 4
#endif
constexpr int DET_WAVES = VSFE_DET_WAVES;
constexpr int DET_THREADS = 64 * DET_WAVES;
constexpr int DET_MAX_TILE_H = 8 * DET_WAVES;
constexpr int DET_MAX_CELLS_Y = DET_WAVES;

// Detector work item: a rectangle of whole cells of one level, with the
// level's geometry copied in (one 64-byte scalar load per block, no
// dependent load of the level record).
struct DetItem {
    int32_t level, cx0, cy0, nkx, nky;           // 32-bit fields: scalar loads only
    int32_t w, h, pitch, cell, ncx;
    int64_t offset, cell_offset, crf_offset;
};
static_assert(sizeof(DetItem) == 64, "DetItem layout");

// Aggregation work item: PYCA_CHUNK consecutive cells of one level.
constexpr int PYCA_CHUNK = 256;
struct CellChunk {
    uint16_t image, level;
    uint32_t first;        // cell index within the level
};

// Byte stride of a column of the smoothed 31 x 31 patch the descriptor tests
// read: point (u, v) of the pattern is at (15 + u) * ORB_PATCH_STRIDE + 15 + v.
constexpr int ORB_PATCH_STRIDE = 36;

// Rotation and bin tables (Q14) of the orientation and rBRIEF steps.
struct OrbTables {
    int32_t bin_x[30], bin_y[30];
};

}  // namespace vsfe

struct vsfe_ctx {
    vsfe_params p;
    int device;
    int tile_w, tile_h;
    uint32_t *d_pattern_off;   // [30][256] rotated test pairs as patch offsets a | b << 16 (device)
    vsfe::OrbTables tables;    // host copy, passed by value to kernels
    int32_t scale_q16[VSFE_MAX_LEVELS];
    int32_t cell[VSFE_MAX_LEVELS];
};

struct vsfe_batch {
    const vsfe_ctx *ctx = nullptr;
    int32_t n_images = 0;
    vsfe_batch_info info{};
    std::vector<vsfe::ImageDev> images;          // host copy
    vsfe::ImageDev *d_images = nullptr;          // device copy
    // pyramid work: items of level l are [pyr_start[l], pyr_start[l+1])
    std::vector<int32_t> pyr_start;
    std::vector<vsfe::PyrItem> h_pyr_items;
    vsfe::PyrItem *d_pyr_items = nullptr;
    // single-launch pyramid: plans, tables (entry = window-local source
    // index | weight << 16), items; twr_lds = dynamic LDS bytes of a block
    int32_t pyr_schedule = 0;                    // VSFE_PYR_* as set (AUTO by default)
    bool twr_ok = false;                         // plan fits (single launch available)
    int32_t twr_tw = 0, twr_th = 0;              // owned level-1 tile of the plan
    int32_t twr_def_w = 0, twr_def_h = 0;        // the batch's default tile (chosen at planning)
    int32_t twr_tab_cap = 0, twr_lds = 0;
    std::vector<vsfe::TowerAxis> h_twr_axes;
    std::vector<uint32_t> h_twr_tab;
    std::vector<vsfe::TowerItem> h_twr_items;
    vsfe::TowerAxis *d_twr_axes = nullptr;
    uint32_t *d_twr_tab = nullptr;
    vsfe::TowerItem *d_twr_items = nullptr;
    // resampling tables: entry = source index | (weight << 16), weight 0 at the far edge
    std::vector<uint32_t> h_coord;
    uint32_t *d_coord = nullptr;
    bool aligned_input = true;                   // level-0 rows start on 4-byte boundaries
    bool aligned_input16 = true;                 // ... and on 16-byte boundaries
    // detector work: per-level tile extents (pixels), items level-major,
    // items of level l are [det_start[l], det_start[l+1])
    int32_t tile_w[VSFE_MAX_LEVELS] = {}, tile_h[VSFE_MAX_LEVELS] = {};
    std::vector<int32_t> det_start;
    int32_t n_det_items = 0;
    std::vector<vsfe::DetItem> h_det_items;
    vsfe::DetItem *d_det_items = nullptr;
    int32_t n_chunks = 0;
    std::vector<vsfe::CellChunk> h_chunks;
    vsfe::CellChunk *d_chunks = nullptr;
    uint8_t *d_run = nullptr;                    // per-cell run flags of the gated detector
    // gated detector work list: [0] = count, then the indices of the items
    // (of the launched level range) with at least one running cell
    int32_t *d_item_list = nullptr;
    int32_t item_list_cap = 0;
    int32_t n_row_tab = 0;                       // stereo: first keypoint of every cell row
    int32_t *d_row_tab = nullptr;
    bool pairs_ok = false;                       // even count, equal pair sizes
    void *cnn = nullptr;                         // proposer plan (levels >= 4)
    vsfe_cnn_info info_cnn{};
};

namespace vsfe {

// A matrix-core product read by ordinary vector instructions: eight more
// wait states between the product and its first reader than the compiler
// inserts.  (With the VGPR-destination forms its count was measured short
// on gfx950: float16 products read right after it were now and then stale
// in their later output columns, varying from run to run.)  The asm takes
// the value as an operand, so it sits between the product and its uses.
template <typename T>
__device__ __forceinline__ T mfma_settle(T v) {
    asm volatile("s_nop 7" : "+v"(v));
    return v;
}

// XCD-aware block order.  Workgroups are dispatched round-robin over the 8
// XCDs (block b runs on XCD b % 8), each with its own L2; this maps block b
// to work item index so that each XCD gets a contiguous range of items
// (neighbouring tiles share halo rows and cache lines in one L2).  A
// bijection on [0, n).
constexpr int N_XCD = 8;
// (Unsigned arithmetic: block indices and counts are never negative, and
// unsigned division by a power of two is a plain shift.)
__device__ __forceinline__ int xcd_item(int b, int n) {
    const unsigned ub = (unsigned)b, un = (unsigned)n;
    const unsigned q = un / N_XCD, r = un % N_XCD;
    const unsigned x = ub % N_XCD, k = ub / N_XCD;
    return (int)((x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k);
}

// XCD-aware order that keeps the dispatch order: groups of G consecutive
// items rotate over the XCDs (group g runs on XCD g % 8), so every XCD
// walks through the whole item list at the same pace (no XCD is left with
// only the heavy first part), while G neighbouring items share one L2.
// Items past the last whole round of 8 G map to themselves.  A bijection on
// [0, n).
template <int G>
__device__ __forceinline__ int xcd_group_item(int b, int n) {
    const unsigned ub = (unsigned)b, un = (unsigned)n;
    const unsigned full = un / (N_XCD * G) * (N_XCD * G);
    if (ub >= full) return b;
    const unsigned x = ub % N_XCD, k = ub / N_XCD;
    return (int)(((k / G) * N_XCD + x) * G + k % G);
}

void set_error(const std::string &msg);
int32_t fail(int32_t code, const std::string &msg);
int32_t check_launch(const char *what);
int32_t check_common(const vsfe_ctx *ctx, const vsfe_batch *b, int32_t *status);

// proposer geometry of a batch (no-op below 4 levels) and its release;
// cnn_plan_check: ECAPACITY when the proposer's 32-bit tables would overflow
// single-launch pyramid plan of a batch (host, after the resampling tables)
// for an owned level-1 tile of tw x th; false if a block would not fit
bool tower_plan(vsfe_batch *b, int tw, int th);
// schedule pyramid_build uses (VSFE_PYR_LEVELS or VSFE_PYR_TOWER)
int32_t pyr_schedule_resolved(const vsfe_batch *b);
// upload the plan (freeing any previous one)
int32_t tower_upload(vsfe_batch *b);
void tower_release(vsfe_batch *b);
int32_t cnn_plan_check(const vsfe_batch *b);
int32_t cnn_setup(vsfe_batch *b);
void cnn_release(vsfe_batch *b);

// detector tiles of one level for a target extent (whole cells, at least one)
void det_items_level(const vsfe_batch *b, int level, int tile_w, int tile_h, std::vector<DetItem> *out);
// rebuild every level's detector items from b->tile_w / b->tile_h (host only)
void det_items_build(vsfe_batch *b);
// (re)allocate the gated detector's work list for the current item count
int32_t det_list_alloc(vsfe_batch *b);
// launch the detector over n device items (no argument checks)
// (item_list: nullable gated work list, [0] = count, then item indices)
int32_t detect_launch(const vsfe_ctx *ctx, const vsfe_batch *b, const DetItem *items, int32_t n_items,
                      const uint8_t *images, const uint8_t *pyr, const uint8_t *cell_mask, uint32_t *cell_keys,
                      uint16_t *crf_debug, const int32_t *item_list, hipStream_t st);

// one-time upload of the orientation disc tables to the current device
int32_t orb_prepare(int device);
// one-time lookup of the aggregation scratch's address on the current device
int32_t pyca_prepare(int device);

// level geometry shared by the host planner
void level_size(int32_t W, int32_t H, int32_t l, int32_t *Wl, int32_t *Hl);
int32_t cell_size(int32_t cell0, int32_t l);
int32_t scale_q16(int32_t l);

}  // namespace vsfe
