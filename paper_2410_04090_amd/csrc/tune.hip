// Detector tile planning and the batch autotuner.
//
// The detector takes one rectangle of whole cells per 256-thread block.  A
// tile shape trades halo overhead (6 extra rows and columns per tile) and
// per-block fixed cost against the number of blocks in flight, and the best
// trade differs per pyramid level because the cell side shrinks from 32 to 8
// pixels.  The autotuner times every distinct whole-cell shape that fits the
// detector's 128 x 32 pixel tile on the batch's own data, level by level,
// and keeps the fastest.  Results never depend on the shape: cells are
// reduced inside one block.
#include <string.h>

#include <algorithm>

#include "vsfe_internal.h"

namespace vsfe {

static void cells_per_tile(int tile_w, int tile_h, int cell, int *nkx, int *nky) {
    *nkx = std::min(32, std::max(1, tile_w / cell));
    *nky = std::min(DET_MAX_CELLS_Y, std::max(1, tile_h / cell));   // at most 32 x DET_WAVES cells (detector LDS)
}

void det_items_level(const vsfe_batch *b, int level, int tile_w, int tile_h, std::vector<DetItem> *out) {
    for (int i = 0; i < b->n_images; i++) {
        const LevelDev &lv = b->images[i].lv[level];
        int nkx, nky;
        cells_per_tile(tile_w, tile_h, lv.cell, &nkx, &nky);
        for (int cy = 0; cy < lv.ncy; cy += nky)
            for (int cx = 0; cx < lv.ncx; cx += nkx)
                out->push_back(DetItem{level, cx, cy, std::min(nkx, lv.ncx - cx), std::min(nky, lv.ncy - cy),
                                       lv.w, lv.h, lv.pitch, lv.cell, lv.ncx, lv.offset, lv.cell_offset,
                                       lv.crf_offset});
    }
}

void det_items_build(vsfe_batch *b) {
    const int L = b->info.n_levels;
    b->h_det_items.clear();
    b->det_start.assign(L + 1, 0);
    for (int l = 0; l < L; l++) {
        b->det_start[l] = (int32_t)b->h_det_items.size();
        det_items_level(b, l, b->tile_w[l], b->tile_h[l], &b->h_det_items);
    }
    b->det_start[L] = (int32_t)b->h_det_items.size();
    b->n_det_items = (int32_t)b->h_det_items.size();
    b->info.n_det_items = b->n_det_items;
}

static bool tile_ok(int tw, int th) { return tw >= 8 && tw <= 128 && th >= 8 && th <= DET_MAX_TILE_H; }

static int32_t upload_items(const std::vector<DetItem> &v, DetItem **dst) {
    *dst = nullptr;
    if (v.empty()) return VSFE_OK;
    if (hipMalloc((void **)dst, v.size() * sizeof(DetItem)) != hipSuccess)
        return fail(VSFE_EHIP, "hipMalloc of detector items failed");
    if (hipMemcpy(*dst, v.data(), v.size() * sizeof(DetItem), hipMemcpyHostToDevice) != hipSuccess)
        return fail(VSFE_EHIP, "upload of detector items failed");
    return VSFE_OK;
}

int32_t det_list_alloc(vsfe_batch *b) {
    if (b->item_list_cap >= b->n_det_items && b->d_item_list) return VSFE_OK;
    int32_t *d = nullptr;
    if (hipMalloc((void **)&d, ((size_t)b->n_det_items + 1) * sizeof(int32_t)) != hipSuccess)
        return fail(VSFE_EHIP, "hipMalloc of the gated work list failed");
    if (b->d_item_list) (void)hipFree(b->d_item_list);
    b->d_item_list = d;
    b->item_list_cap = b->n_det_items;
    return VSFE_OK;
}

// Replace the device item table after b->tile_w / b->tile_h changed.
static int32_t det_items_refresh(vsfe_batch *b) {
    det_items_build(b);
    DetItem *d = nullptr;
    int32_t rc = upload_items(b->h_det_items, &d);
    if (rc) return rc;
    if (b->d_det_items) (void)hipFree(b->d_det_items);
    b->d_det_items = d;
    return det_list_alloc(b);
}

// Pyramid schedule pass of the autotuner: the batch's current schedule
// first (the baseline), then one launch per level and single-launch tiles
// from small (more blocks, more halo) to large; tiles whose block does not
// fit are skipped.  The fastest is installed.
static int32_t tune_pyramid(const vsfe_ctx *ctx, vsfe_batch *b, const uint8_t *images, uint8_t *pyr,
                            int32_t *status, int reps, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                            vsfe_tune_report *out) {
    struct Cand { int s, tw, th; };
    int32_t s0, tw0, th0;
    int32_t rc = vsfe_batch_pyramid_get(b, &s0, &tw0, &th0);
    if (rc) return rc;
    std::vector<Cand> cand{{s0, tw0, th0}};
    if (s0 != VSFE_PYR_LEVELS) cand.push_back({VSFE_PYR_LEVELS, tw0, th0});
    static const int kT[][2] = {{48, 8}, {64, 16}, {96, 24}, {112, 32}, {112, 48}, {160, 32}, {200, 24}, {240, 32}};
    for (const auto &t : kT)
        if (!(s0 == VSFE_PYR_TOWER && t[0] == tw0 && t[1] == th0)) cand.push_back({VSFE_PYR_TOWER, t[0], t[1]});
    float best = 0.f;
    int best_k = -1, tried = 0;
    float worst = 0.f;
    for (size_t k = 0; k < cand.size(); k++) {
        rc = vsfe_batch_set_pyramid(b, cand[k].s, cand[k].tw, cand[k].th);
        if (rc == VSFE_ECAPACITY) continue;   // this tile's block does not fit
        if (rc) return rc;
        rc = pyramid_build(ctx, b, images, pyr, status, st);   // warm-up
        if (rc) return rc;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && !rc; r++) rc = pyramid_build(ctx, b, images, pyr, status, st);
        (void)hipEventRecord(e1, st);
        if (rc) return rc;
        if (hipEventSynchronize(e1) != hipSuccess) return fail(VSFE_EHIP, "tuning run failed");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const float us = ms * 1000.f / reps;
        tried++;
        if (k == 0) out->pyr_us_before = us;
        worst = std::max(worst, us);
        if (best_k < 0 || us < best) {
            best = us;
            best_k = (int)k;
        }
    }
    if (best_k < 0) return fail(VSFE_EHIP, "no pyramid schedule could be timed");
    rc = vsfe_batch_set_pyramid(b, cand[best_k].s, cand[best_k].tw, cand[best_k].th);
    if (rc) return rc;
    out->pyr_schedule = cand[best_k].s;
    out->pyr_tile_w = cand[best_k].tw;
    out->pyr_tile_h = cand[best_k].th;
    out->pyr_us = best;
    out->pyr_us_worst = worst;
    out->pyr_n_tried = tried;
    return VSFE_OK;
}

}  // namespace vsfe

using namespace vsfe;

extern "C" {

int32_t vsfe_batch_tiles_get(const vsfe_batch *b, int32_t *tile_w, int32_t *tile_h) {
    if (!b || !tile_w || !tile_h) return fail(VSFE_EINVAL, "null argument");
    for (int l = 0; l < b->info.n_levels; l++) {
        tile_w[l] = b->tile_w[l];
        tile_h[l] = b->tile_h[l];
    }
    return VSFE_OK;
}

int32_t vsfe_batch_set_tiles(vsfe_batch *b, const int32_t *tile_w, const int32_t *tile_h) {
    if (!b || !tile_w || !tile_h) return fail(VSFE_EINVAL, "null argument");
    for (int l = 0; l < b->info.n_levels; l++)
        if (!tile_ok(tile_w[l], tile_h[l])) return fail(VSFE_EINVAL, "tile out of range at level " + std::to_string(l));
    if (hipDeviceSynchronize() != hipSuccess) return fail(VSFE_EHIP, "device synchronisation failed");
    for (int l = 0; l < b->info.n_levels; l++) {
        b->tile_w[l] = tile_w[l];
        b->tile_h[l] = tile_h[l];
    }
    return det_items_refresh(b);
}

int32_t vsfe_batch_autotune(const vsfe_ctx *ctx, vsfe_batch *b, const uint8_t *images, const uint8_t *pyr,
                            uint32_t *cell_keys, int32_t *status, int32_t reps, void *stream,
                            vsfe_tune_report *out) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !cell_keys || !out || (!pyr && b->info.n_levels > 1)) return fail(VSFE_EINVAL, "null argument");
    if (reps < 1 || reps > 1000) return fail(VSFE_EINVAL, "reps must be in 1..1000");
    hipStream_t st = (hipStream_t)stream;
    const int L = b->info.n_levels;
    memset(out, 0, sizeof(*out));
    out->n_levels = L;
    static const int kW[] = {16, 24, 32, 40, 48, 64, 80, 96, 112, 128};
    static const int kH[] = {8, 12, 16, 24, 32, 48, 64};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(VSFE_EHIP, "hipEventCreate failed");
    if (L > 1) {
        // the rebuilt pyramid is byte-identical whatever the schedule
        rc = tune_pyramid(ctx, b, images, const_cast<uint8_t *>(pyr), status, reps, st, e0, e1, out);
        if (rc) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rc;
        }
    }
    DetItem *d_items = nullptr;
    size_t cap = 0;
    for (int l = 0; l < L && !rc; l++) {
        const int c = b->images[0].lv[l].cell;
        // candidate shapes: distinct (cells across, cells down); the batch's
        // current shape first so that its time is reported as the baseline
        std::vector<std::pair<int, int>> cand{{b->tile_w[l], b->tile_h[l]}};
        std::vector<std::pair<int, int>> seen;
        int nx0, ny0;
        cells_per_tile(b->tile_w[l], b->tile_h[l], c, &nx0, &ny0);
        seen.push_back({nx0, ny0});
        for (int tw : kW)
            for (int th : kH) {
                if (th > DET_MAX_TILE_H) continue;
                int nx, ny;
                cells_per_tile(tw, th, c, &nx, &ny);
                if (std::find(seen.begin(), seen.end(), std::make_pair(nx, ny)) != seen.end()) continue;
                seen.push_back({nx, ny});
                cand.push_back({tw, th});
            }
        float best = 0.f;
        int best_k = 0;
        std::vector<float> times;
        for (size_t k = 0; k < cand.size() && !rc; k++) {
            std::vector<DetItem> items;
            det_items_level(b, l, cand[k].first, cand[k].second, &items);
            if (items.size() > cap) {
                if (d_items) (void)hipFree(d_items);
                d_items = nullptr;
                if (hipMalloc((void **)&d_items, items.size() * sizeof(DetItem)) != hipSuccess) {
                    rc = fail(VSFE_EHIP, "hipMalloc of tuning items failed");
                    break;
                }
                cap = items.size();
            }
            if (hipMemcpy(d_items, items.data(), items.size() * sizeof(DetItem), hipMemcpyHostToDevice) != hipSuccess) {
                rc = fail(VSFE_EHIP, "upload of tuning items failed");
                break;
            }
            const int n = (int)items.size();
            rc = detect_launch(ctx, b, d_items, n, images, pyr, nullptr, cell_keys, nullptr, nullptr, st);   // warm-up
            if (rc) break;
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < reps && !rc; r++)
                rc = detect_launch(ctx, b, d_items, n, images, pyr, nullptr, cell_keys, nullptr, nullptr, st);
            (void)hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) rc = fail(VSFE_EHIP, "tuning run failed");
            if (rc) break;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const float us = ms * 1000.f / reps;
            if (k == 0) out->us_before[l] = us;
            times.push_back(us);
            if (k == 0 || us < best) {
                best = us;
                best_k = (int)k;
            }
        }
        int nx, ny;
        cells_per_tile(cand[best_k].first, cand[best_k].second, c, &nx, &ny);
        // store the extent actually used (whole cells) so that every image of
        // the batch gets the same cell counts
        b->tile_w[l] = std::min(128, std::max(8, nx * c));
        b->tile_h[l] = std::min(DET_MAX_TILE_H, std::max(8, ny * c));
        out->tile_w[l] = nx * c;
        out->tile_h[l] = ny * c;
        out->us[l] = best;
        out->n_tried[l] = (int32_t)cand.size();
        if (!times.empty()) {
            std::sort(times.begin(), times.end());
            out->us_worst[l] = times.back();
            out->us_median[l] = times[times.size() / 2];
        }
    }
    if (d_items) (void)hipFree(d_items);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    return det_items_refresh(b);
}

}  // extern "C"
