// Host side of the gfx950 front-end library: parameters, level geometry,
// context (constant tables), batch planner (device work tables), errors.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "vsfe_internal.h"

namespace vsfe {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int32_t fail(int32_t code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int32_t check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VSFE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return VSFE_OK;
}

int32_t check_common(const vsfe_ctx *ctx, const vsfe_batch *b, int32_t *status) {
    (void)status;
    if (!ctx || !b) return fail(VSFE_EINVAL, "null context or batch");
    if (b->ctx != ctx) return fail(VSFE_EINVAL, "batch was created with another context");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device)
        return fail(VSFE_EINVAL, "current HIP device differs from the context's device");
    return VSFE_OK;
}

static int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

// W_l = floor(W / 1.2^l + 1/2) in exact integers.
void level_size(int32_t W, int32_t H, int32_t l, int32_t *Wl, int32_t *Hl) {
    const int64_t num = ipow(5, l), den = ipow(6, l);
    *Wl = (int32_t)((2 * (int64_t)W * num + den) / (2 * den));
    *Hl = (int32_t)((2 * (int64_t)H * num + den) / (2 * den));
}

// 32-pixel native cells shrink to 8 pixels at the eighth level (Sec. IV-F).
int32_t cell_size(int32_t cell0, int32_t l) { return (int32_t)(((int64_t)cell0 * ipow(5, l)) / ipow(6, l)); }

// round(65536 * 1.2^l)
int32_t scale_q16(int32_t l) {
    const int64_t num = 65536 * ipow(6, l), den = ipow(5, l);
    return (int32_t)((2 * num + den) / (2 * den));
}

}  // namespace vsfe
extern "C" int32_t vsfe_params_check(const vsfe_params *p);
namespace vsfe {
static int32_t params_check_impl(const vsfe_params *p) { return vsfe_params_check(p); }

static int32_t round_half_away(int64_t a) {
    const int64_t m = a < 0 ? -a : a;
    const int64_t r = (m + 8192) >> 14;
    return (int32_t)(a < 0 ? -r : r);
}

template <class T>
static int32_t upload(const std::vector<T> &v, T **dst) {
    *dst = nullptr;
    if (v.empty()) return VSFE_OK;
    if (hipMalloc((void **)dst, v.size() * sizeof(T)) != hipSuccess) return fail(VSFE_EHIP, "hipMalloc of a work table failed");
    if (hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return fail(VSFE_EHIP, "upload of a work table failed");
    return VSFE_OK;
}


// Host-only planning of a batch: level geometry, buffer sizes, work items.
static int32_t plan_batch(const vsfe_params &p, int tile_w, int tile_h, int32_t n,
                          const int32_t *widths, const int32_t *heights, const int32_t *pitches,
                          const int64_t *offsets, vsfe_batch *b) {
    if (!widths || !heights || !pitches || !offsets) return fail(VSFE_EINVAL, "null argument");
    if (n < 1) return fail(VSFE_EINVAL, "empty batch");
    if (n > VSFE_MAX_IMAGES) return fail(VSFE_ECAPACITY, "too many images in one batch");
    int32_t rc = params_check_impl(&p);
    if (rc) return rc;
    const int L = p.n_levels;
    b->n_images = n;
    b->images.resize(n);
    memset(&b->info, 0, sizeof(b->info));
    b->info.n_images = n;
    b->info.n_levels = L;

    int64_t cell_at = 0, crf_at = 0, cell0_at = 0, pyr_at = 0, in_end = 0, row_at = 0;
    for (int i = 0; i < n; i++) {
        const int W = widths[i], H = heights[i];
        if (W < 1 || H < 1 || W > VSFE_MAX_DIM || H > VSFE_MAX_DIM || pitches[i] < W || offsets[i] < 0)
            return fail(VSFE_EINVAL, "image " + std::to_string(i) + ": bad size, pitch or offset");
        in_end = std::max(in_end, offsets[i] + (int64_t)pitches[i] * H);
        ImageDev &im = b->images[i];
        memset(&im, 0, sizeof(im));
        im.w = W;
        im.h = H;
        im.n_levels = L;
        im.cell_base = cell_at;
        im.cell0_offset = cell0_at;
        im.kp_offset = (int64_t)i * p.n_max;
        for (int l = 0; l < L; l++) {
            LevelDev &lv = im.lv[l];
            level_size(W, H, l, &lv.w, &lv.h);
            if (lv.w < 1 || lv.h < 1)
                return fail(VSFE_EINVAL, "image " + std::to_string(i) + ": level " + std::to_string(l) + " is empty");
            lv.cell = cell_size(p.cell0, l);
            lv.ncx = (lv.w + lv.cell - 1) / lv.cell;
            lv.ncy = (lv.h + lv.cell - 1) / lv.cell;
            lv.scale_q16 = scale_q16(l);
            if (l == 0) {
                lv.pitch = pitches[i];
                lv.offset = offsets[i];
            } else {
                lv.pitch = (lv.w + 63) & ~63;
                lv.offset = pyr_at;
                pyr_at += ((int64_t)lv.pitch * lv.h + 255) & ~(int64_t)255;
            }
            lv.cell_offset = cell_at;
            lv.crf_offset = crf_at;
            lv.row_tab = (int32_t)row_at;
            row_at += lv.ncy;
            cell_at += (int64_t)lv.ncx * lv.ncy;
            crf_at += (int64_t)lv.w * lv.h;
        }
        im.row_tab_end = (int32_t)row_at;
        row_at += 1;                             // the entry after the last cell row
        im.n_cells = cell_at - im.cell_base;
        cell0_at += (int64_t)im.lv[0].ncx * im.lv[0].ncy;
    }
    // the proposer's 32-bit prefix tables must hold the batch (before any
    // per-tile work list is built)
    rc = cnn_plan_check(b);
    if (rc) return rc;
    // resampling tables, one per distinct (source size, level): entry o holds
    // the floored Q8 source coordinate of output o (index | weight << 16),
    // weight forced to 0 where the right / bottom neighbour is clamped
    b->h_coord.clear();
    b->aligned_input = true;
    b->aligned_input16 = true;
    for (int i = 0; i < n; i++) {
        if ((pitches[i] & 3) || (offsets[i] & 3)) b->aligned_input = false;
        if ((pitches[i] & 15) || (offsets[i] & 15)) b->aligned_input16 = false;
    }
    auto q8 = [](int64_t o, int64_t n_src, int64_t n_dst, int *a, int *f) {
        const int64_t t = ((2 * o + 1) * n_src - n_dst) * 128 / n_dst;
        *a = (int)(t >> 8);
        *f = (int)(t & 255);
        if (*a + 1 >= n_src) *f = 0;
    };
    std::vector<std::pair<std::pair<int, int>, int>> seen;   // ((W, H), image with its tables)
    for (int i = 0; i < n; i++) {
        ImageDev &im = b->images[i];
        int from = -1;
        for (auto &sv : seen)
            if (sv.first.first == im.w && sv.first.second == im.h) from = sv.second;
        if (from >= 0) {
            for (int l = 1; l < L; l++) {
                im.lv[l].xtab = b->images[from].lv[l].xtab;
                im.lv[l].ytab = b->images[from].lv[l].ytab;
            }
            continue;
        }
        seen.push_back({{im.w, im.h}, i});
        for (int l = 1; l < L; l++) {
            const LevelDev &s = im.lv[l - 1];
            LevelDev &d = im.lv[l];
            d.xtab = (int32_t)b->h_coord.size();
            for (int o = 0; o < d.w; o++) {
                int a, f;
                q8(o, s.w, d.w, &a, &f);
                b->h_coord.push_back((uint32_t)a | ((uint32_t)f << 16));
            }
            d.ytab = (int32_t)b->h_coord.size();
            for (int o = 0; o < d.h; o++) {
                int a, f;
                q8(o, s.h, d.h, &a, &f);
                b->h_coord.push_back((uint32_t)a | ((uint32_t)f << 16));
            }
        }
    }
    // pyramid tiles, level-major so that one launch covers one level of all
    // images; each records the source window it reads
    b->pyr_start.assign(L + 1, 0);
    b->h_pyr_items.clear();
    for (int l = 1; l < L; l++) {
        b->pyr_start[l] = (int32_t)b->h_pyr_items.size();
        for (int i = 0; i < n; i++) {
            const LevelDev &s = b->images[i].lv[l - 1];
            const LevelDev &lv = b->images[i].lv[l];
            for (int ty = 0; ty < (lv.h + PYR_TH - 1) / PYR_TH; ty++)
                for (int tx = 0; tx < (lv.w + PYR_TW - 1) / PYR_TW; tx++) {
                    const int ox0 = tx * PYR_TW, ox1 = std::min(lv.w, ox0 + PYR_TW) - 1;
                    const int oy0 = ty * PYR_TH, oy1 = std::min(lv.h, oy0 + PYR_TH) - 1;
                    const int xa0 = (int)(b->h_coord[lv.xtab + ox0] & 0xFFFF) & ~15;
                    const int xa1 = (int)(b->h_coord[lv.xtab + ox1] & 0xFFFF) + 1;
                    const int ya0 = (int)(b->h_coord[lv.ytab + oy0] & 0xFFFF);
                    const int ya1 = (int)(b->h_coord[lv.ytab + oy1] & 0xFFFF) + 1;
                    const int ncols = ((xa1 - xa0 + 1) + 15) & ~15, nrows = ya1 - ya0 + 1;
                    if (ncols > PYR_SW || nrows > PYR_SH)
                        return fail(VSFE_ECAPACITY, "pyramid source window exceeds the staging buffer");
                    b->h_pyr_items.push_back(PyrItem{s.offset, lv.offset, s.w, s.h, s.pitch, lv.w, lv.h, lv.pitch,
                                                     lv.xtab, lv.ytab, tx, ty, xa0, ya0, ncols, nrows});
                }
        }
    }
    b->pyr_start[L] = (int32_t)b->h_pyr_items.size();
    // single-launch schedule at the default tile (unavailable if a block
    // would not fit: the per-level schedule is then the only one)
    b->twr_ok = tower_plan(b, TWR_TW, TWR_TH);
    if (b->twr_ok && (int)b->h_twr_items.size() < TWR_SMALL_ITEMS && !tower_plan(b, 64, 16))
        b->twr_ok = tower_plan(b, TWR_TW, TWR_TH);
    b->twr_def_w = b->twr_tw;
    b->twr_def_h = b->twr_th;
    // detector tiles: whole cells, about tile_w x tile_h pixels at every level
    for (int l = 0; l < L; l++) {
        b->tile_w[l] = tile_w;
        b->tile_h[l] = tile_h;
    }
    det_items_build(b);
    b->h_chunks.clear();
    for (int i = 0; i < n; i++)
        for (int l = 0; l < L; l++) {
            const LevelDev &lv = b->images[i].lv[l];
            const int64_t nc = (int64_t)lv.ncx * lv.ncy;
            for (int64_t s = 0; s < nc; s += PYCA_CHUNK)
                b->h_chunks.push_back(CellChunk{(uint16_t)i, (uint16_t)l, (uint32_t)s});
        }
    b->pairs_ok = (n % 2 == 0);
    for (int i = 0; b->pairs_ok && i + 1 < n; i += 2)
        if (widths[i] != widths[i + 1] || heights[i] != heights[i + 1]) b->pairs_ok = false;

    b->info.input_bytes = in_end;
    b->info.pyr_bytes = std::max<int64_t>(pyr_at, 256);
    b->info.crf_elems = crf_at;
    b->info.n_cells = cell_at;
    b->n_row_tab = (int32_t)row_at;
    b->info.n_cells0 = cell0_at;
    b->info.kp_capacity = (int64_t)n * p.n_max;
    b->info.workspace_bytes = cell_at * 4 + 256;
    b->info.match_capacity = (int64_t)(n / 2) * p.n_max;
    b->n_det_items = (int32_t)b->h_det_items.size();
    b->n_chunks = (int32_t)b->h_chunks.size();
    return VSFE_OK;
}

}  // namespace vsfe

using namespace vsfe;

extern "C" {

const char *vsfe_last_error(void) { return g_last_error.c_str(); }

void vsfe_params_default(vsfe_params *p) {
    if (!p) return;
    p->eps_hi = 20;
    p->eps_lo = 7;
    p->p_min = 9;
    p->p_max = 13;
    p->border = 16;
    p->n_levels = 8;
    p->cell0 = 32;
    p->pfa = 1;
    p->nms_mode = 0;
    p->nms_radius = 1;
    p->n_max = 2000;
    p->blur = 1;
    p->d_max = 96;
    p->match_th = 64;
    p->row_band = 1;
}

int32_t vsfe_params_check(const vsfe_params *p) {
    if (!p) return fail(VSFE_EINVAL, "null params");
    if (p->eps_hi < 0 || p->eps_hi > 254) return fail(VSFE_EINVAL, "eps_hi out of 0..254");
    if (p->eps_lo < -1 || p->eps_lo > p->eps_hi) return fail(VSFE_EINVAL, "eps_lo must be -1 or 0..eps_hi");
    if (p->p_min < 1 || p->p_min > 16 || p->p_max < p->p_min || p->p_max > 16)
        return fail(VSFE_EINVAL, "need 1 <= p_min <= p_max <= 16");
    if (p->border < 3 || p->border > 64) return fail(VSFE_EINVAL, "border out of 3..64");
    if (p->n_levels < 1 || p->n_levels > VSFE_MAX_LEVELS) return fail(VSFE_EINVAL, "n_levels out of range");
    // a detector tile holds at least one whole cell (DET_MAX_TILE_H = 32 rows)
    if (p->cell0 < 8 || p->cell0 > DET_MAX_TILE_H) return fail(VSFE_EINVAL, "cell0 out of 8..32");
    if (cell_size(p->cell0, p->n_levels - 1) < 1) return fail(VSFE_EINVAL, "cell side vanishes at the last level");
    if (p->pfa != 0 && p->pfa != 1) return fail(VSFE_EINVAL, "pfa must be 0 or 1");
    if (p->nms_mode != 0 && p->nms_mode != 1) return fail(VSFE_EINVAL, "nms_mode must be 0 or 1");
    if (p->nms_radius < 0 || p->nms_radius > 3) return fail(VSFE_EINVAL, "nms_radius out of 0..3");
    if (p->n_max < 1 || p->n_max > 65535) return fail(VSFE_EINVAL, "n_max out of 1..65535");
    if (p->blur != 0 && p->blur != 1) return fail(VSFE_EINVAL, "blur must be 0 or 1");
    if (p->d_max < 0 || p->d_max > 4096) return fail(VSFE_EINVAL, "d_max out of 0..4096");
    if (p->match_th < 0 || p->match_th > 256) return fail(VSFE_EINVAL, "match_th out of 0..256");
    if (p->row_band < 0 || p->row_band > 3) return fail(VSFE_EINVAL, "row_band out of 0..3");
    return VSFE_OK;
}

int32_t vsfe_level_geometry(const vsfe_params *p, int32_t W, int32_t H, int32_t level,
                            int32_t *Wl, int32_t *Hl, int32_t *cell) {
    if (!p || !Wl || !Hl || !cell) return fail(VSFE_EINVAL, "null argument");
    if (W < 1 || H < 1 || W > VSFE_MAX_DIM || H > VSFE_MAX_DIM) return fail(VSFE_EINVAL, "image size out of range");
    if (level < 0 || level >= VSFE_MAX_LEVELS) return fail(VSFE_EINVAL, "level out of range");
    level_size(W, H, level, Wl, Hl);
    *cell = cell_size(p->cell0, level);
    return VSFE_OK;
}

int32_t vsfe_ctx_create(const vsfe_params *p, const int8_t *pattern, vsfe_ctx **out) {
    if (!out) return fail(VSFE_EINVAL, "null output pointer");
    *out = nullptr;
    int32_t rc = vsfe_params_check(p);
    if (rc) return rc;
    if (!pattern) return fail(VSFE_EINVAL, "null pattern");
    for (int t = 0; t < 256; t++)
        for (int e = 0; e < 2; e++) {
            const int u = pattern[4 * t + 2 * e], v = pattern[4 * t + 2 * e + 1];
            if (u * u + v * v > 225) return fail(VSFE_EINVAL, "pattern point outside the radius-15 disc");
        }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(VSFE_EUNSUPPORTED, "no HIP device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(VSFE_EHIP, "hipGetDeviceProperties failed");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(VSFE_EUNSUPPORTED, std::string("library built for gfx950, device is ") + prop.gcnArchName);

    rc = orb_prepare(dev);
    if (rc) return rc;
    rc = pyca_prepare(dev);
    if (rc) return rc;
    vsfe_ctx *c = new vsfe_ctx();
    c->p = *p;
    c->device = dev;
    c->tile_w = 128;
    c->tile_h = DET_MAX_TILE_H;
    for (int l = 0; l < VSFE_MAX_LEVELS; l++) {
        c->scale_q16[l] = scale_q16(l);
        c->cell[l] = cell_size(p->cell0, l);
    }
    // Q14 rotation table (12-degree steps) and bin boundaries at 6 + 12 j degrees.
    int32_t C[30], S[30];
    for (int k = 0; k < 30; k++) {
        const double a = (double)k * 12.0 * M_PI / 180.0;
        C[k] = (int32_t)lround(16384.0 * cos(a));
        S[k] = (int32_t)lround(16384.0 * sin(a));
        const double bnd = (6.0 + 12.0 * (double)k) * M_PI / 180.0;
        c->tables.bin_x[k] = (int32_t)lround(16384.0 * cos(bnd));
        c->tables.bin_y[k] = (int32_t)lround(16384.0 * sin(bnd));
    }
    std::vector<uint32_t> rot(30 * 256);
    for (int k = 0; k < 30; k++)
        for (int t = 0; t < 256; t++)
            for (int e = 0; e < 2; e++) {
                const int64_t u = pattern[4 * t + 2 * e], v = pattern[4 * t + 2 * e + 1];
                const int32_t ur = round_half_away(u * C[k] - v * S[k]);
                const int32_t vr = round_half_away(u * S[k] + v * C[k]);
                if (ur < -15 || ur > 15 || vr < -15 || vr > 15) {
                    delete c;
                    return fail(VSFE_EINVAL, "rotated pattern leaves the 31x31 patch");
                }
                rot[k * 256 + t] |= (uint32_t)((15 + ur) * ORB_PATCH_STRIDE + 15 + vr) << (16 * e);
            }
    if (hipMalloc((void **)&c->d_pattern_off, rot.size() * sizeof(uint32_t)) != hipSuccess) {
        delete c;
        return fail(VSFE_EHIP, "hipMalloc of the pattern table failed");
    }
    if (hipMemcpy(c->d_pattern_off, rot.data(), rot.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c->d_pattern_off);
        delete c;
        return fail(VSFE_EHIP, "upload of the pattern table failed");
    }
    *out = c;
    return VSFE_OK;
}

int32_t vsfe_ctx_destroy(vsfe_ctx *ctx) {
    if (!ctx) return VSFE_OK;
    if (ctx->d_pattern_off) (void)hipFree(ctx->d_pattern_off);
    delete ctx;
    return VSFE_OK;
}

int32_t vsfe_ctx_set_tile(vsfe_ctx *ctx, int32_t tile_w, int32_t tile_h) {
    if (!ctx) return fail(VSFE_EINVAL, "null context");
    if (tile_w < 8 || tile_w > 128 || tile_h < 8 || tile_h > DET_MAX_TILE_H) return fail(VSFE_EINVAL, "tile out of range");
    ctx->tile_w = tile_w;
    ctx->tile_h = tile_h;
    return VSFE_OK;
}

int32_t vsfe_batch_destroy(vsfe_batch *b) {
    if (!b) return VSFE_OK;
    if (b->d_images) (void)hipFree(b->d_images);
    if (b->d_pyr_items) (void)hipFree(b->d_pyr_items);
    if (b->d_coord) (void)hipFree(b->d_coord);
    if (b->d_det_items) (void)hipFree(b->d_det_items);
    if (b->d_chunks) (void)hipFree(b->d_chunks);
    if (b->d_run) (void)hipFree(b->d_run);
    if (b->d_item_list) (void)hipFree(b->d_item_list);
    if (b->d_row_tab) (void)hipFree(b->d_row_tab);
    tower_release(b);
    cnn_release(b);
    delete b;
    return VSFE_OK;
}

int32_t vsfe_batch_plan(const vsfe_params *p, int32_t n, const int32_t *widths,
                        const int32_t *heights, const int32_t *pitches, const int64_t *offsets,
                        vsfe_batch_info *out) {
    if (!p || !out) return fail(VSFE_EINVAL, "null argument");
    vsfe_batch tmp;
    int32_t rc = plan_batch(*p, 128, 32, n, widths, heights, pitches, offsets, &tmp);
    if (rc) return rc;
    *out = tmp.info;
    return VSFE_OK;
}

int32_t vsfe_batch_create(const vsfe_ctx *ctx, int32_t n, const int32_t *widths,
                          const int32_t *heights, const int32_t *pitches,
                          const int64_t *offsets, vsfe_batch **out) {
    if (!out) return fail(VSFE_EINVAL, "null output pointer");
    *out = nullptr;
    if (!ctx) return fail(VSFE_EINVAL, "null context");
    vsfe_batch *b = new vsfe_batch();
    b->ctx = ctx;
    int32_t rc = plan_batch(ctx->p, ctx->tile_w, ctx->tile_h, n, widths, heights, pitches, offsets, b);
    if (!rc) rc = upload(b->images, &b->d_images);
    if (!rc) rc = upload(b->h_pyr_items, &b->d_pyr_items);
    if (!rc && b->twr_ok) rc = tower_upload(b);
    if (!rc) rc = upload(b->h_coord, &b->d_coord);
    if (!rc) rc = upload(b->h_det_items, &b->d_det_items);
    if (!rc) rc = upload(b->h_chunks, &b->d_chunks);
    if (!rc && b->info.n_cells > 0 && hipMalloc((void **)&b->d_run, (size_t)b->info.n_cells) != hipSuccess)
        rc = fail(VSFE_EHIP, "hipMalloc of the run-flag table failed");
    if (!rc) rc = det_list_alloc(b);
    if (!rc && b->n_row_tab > 0 &&
        hipMalloc((void **)&b->d_row_tab, (size_t)b->n_row_tab * sizeof(int32_t)) != hipSuccess)
        rc = fail(VSFE_EHIP, "hipMalloc of the row-start table failed");
    if (!rc) rc = cnn_setup(b);
    if (rc) {
        vsfe_batch_destroy(b);
        return rc;
    }
    *out = b;
    return VSFE_OK;
}

int32_t vsfe_batch_info_get(const vsfe_batch *b, vsfe_batch_info *out) {
    if (!b || !out) return fail(VSFE_EINVAL, "null argument");
    *out = b->info;
    return VSFE_OK;
}

int32_t vsfe_batch_level_info(const vsfe_batch *b, int32_t image, int32_t level, vsfe_level_info *out) {
    if (!b || !out) return fail(VSFE_EINVAL, "null argument");
    if (image < 0 || image >= b->n_images || level < 0 || level >= b->info.n_levels)
        return fail(VSFE_EINVAL, "image or level out of range");
    const ImageDev &im = b->images[image];
    const LevelDev &lv = im.lv[level];
    out->width = lv.w;
    out->height = lv.h;
    out->pitch = lv.pitch;
    out->cell = lv.cell;
    out->ncx = lv.ncx;
    out->ncy = lv.ncy;
    out->offset = lv.offset;
    out->cell_offset = lv.cell_offset;
    out->crf_offset = lv.crf_offset;
    out->cell0_offset = im.cell0_offset;
    return VSFE_OK;
}

}  // extern "C"
