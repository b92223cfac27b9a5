// Stereo matching along rectified rows by descriptor-distance minimisation
// (Sec. III-3, the middle-end's stereo matcher).
//
// 1 to 16 lanes per left keypoint.  Right keypoints are stored in canonical
// order (level, cell row, cell column), so the candidates of a left
// keypoint at level l and row y -- same level, |dy| <= row_band -- lie in
// the contiguous run of cell rows floor((y - band) / c_l) ..
// floor((y + band) / c_l).  On batches of at least 16384 keypoint slots a
// first pass writes, for every cell row of every right image, the index of
// its first keypoint (one thread per keypoint fills the rows from the
// previous keypoint's row to its own), so that run is two table reads;
// smaller batches search for the run's start instead (one launch less,
// which is what a single pair's latency is made of).  Each candidate
// with native-scale disparity d = x0_l - x0_r in [0, d_max] costs eight
// popcounts; the least distance wins, ties to smaller |dy|, smaller d,
// smaller index (ascending scan with strict comparisons).
#include "vsfe_internal.h"

namespace vsfe {

struct StereoArgs {
    int cell[VSFE_MAX_LEVELS];
    int n_max, n_pairs, d_max, match_th, band;
};

// Row-start table of the right images: entry lv.row_tab + cy holds the
// index of the first keypoint of cell row cy of level l, or of the next row
// that has one (the rows of all levels are consecutive; entry row_tab_end is
// the keypoint count).  Thread j of image ri writes the entries after the
// previous keypoint's row up to its own row; thread count writes the rest.
__global__ __launch_bounds__(256) void row_table_kernel(const ImageDev *__restrict__ imgs, vsfe_kp_soa kps,
                                                        const int32_t *__restrict__ kp_count,
                                                        int32_t *__restrict__ tab, StereoArgs a) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int pair = (int)(s / (a.n_max + 1));
    const int j = (int)(s - (int64_t)pair * (a.n_max + 1));
    if (pair >= a.n_pairs) return;
    const ImageDev &im = imgs[2 * pair + 1];
    const int nr = kp_count[2 * pair + 1];
    if (j > nr) return;
    auto entry = [&](int k) {               // table entry of keypoint k's cell row
        const int64_t rs = im.kp_offset + k;
        // (clamped into the image's table whatever the arrays hold)
        const int l = min((int)kps.level[rs], im.n_levels - 1);
        return im.lv[l].row_tab + min((int)kps.y[rs] / a.cell[l], im.lv[l].ncy - 1);
    };
    const int lo = j > 0 ? entry(j - 1) + 1 : im.lv[0].row_tab;
    const int hi = j < nr ? entry(j) : im.row_tab_end;
    for (int e = lo; e <= hi; e++) tab[e] = j;
}

// G lanes per left keypoint (1, 4 or 16: more for small batches, whose
// few keypoints leave the GPU waiting on each candidate walk): lane k scans
// candidates start + k, + G, ... and the group keeps the least (distance,
// |dy|, disparity, index) key, which is the ascending scan's choice with
// strict comparisons.  SEARCH (16 lanes, small batches): no row-start
// table; the group finds the first candidate by a 16-way search over the
// right keypoints, and each lane's walk stops at its first keypoint past
// the last candidate row (the same candidates for keypoints in canonical
// order; any order stays inside the image's slots).
template <int ST_GROUP, bool SEARCH>
__global__ __launch_bounds__(256) void stereo_kernel(const ImageDev *__restrict__ imgs, vsfe_kp_soa kps,
                                                     const int32_t *__restrict__ kp_count,
                                                     const uint32_t *__restrict__ desc, int32_t *__restrict__ midx,
                                                     uint16_t *__restrict__ mdist, int16_t *__restrict__ mdisp,
                                                     const int32_t *__restrict__ tab, StereoArgs a) {
    const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / ST_GROUP;
    const int k = threadIdx.x & (ST_GROUP - 1);
    const int pair = (int)(s / a.n_max);
    const int i = (int)(s - (int64_t)pair * a.n_max);
    if (pair >= a.n_pairs) return;                      // (whole groups exit together)
    const int li = 2 * pair, ri = 2 * pair + 1;
    if (i >= kp_count[li]) return;
    const int64_t lslot = imgs[li].kp_offset + i;
    const int64_t rbase = imgs[ri].kp_offset;
    const int nr = kp_count[ri];
    const int level = kps.level[lslot], y = kps.y[lslot], x0 = kps.x0[lslot];
    uint32_t d[8];
#pragma unroll
    for (int w = 0; w < 8; w++) d[w] = desc[lslot * 8 + w];

    const LevelDev &rl = imgs[ri].lv[level];
    const int c = a.cell[level];
    const int cy_lo = max(y - a.band, 0) / c, cy_hi = min((y + a.band) / c, rl.ncy - 1);
    int start, end;
    if constexpr (SEARCH) {
        static_assert(ST_GROUP == 16, "the search takes a group of 16 lanes");
        // first right keypoint at (level, row cy_lo) or after: each step the
        // group probes 16 evenly spaced keypoints of [lo, hi) and keeps the
        // gap after the last one that is still before the target
        int lo = 0, hi = nr;
        const int gshift = (int)(threadIdx.x & 63) & ~(ST_GROUP - 1);
        while (lo < hi) {                                  // (uniform in the group)
            const int step = (hi - lo + ST_GROUP - 1) / ST_GROUP;
            const int p = lo + k * step;
            bool before = false;
            if (p < hi) {
                const int64_t rs = rbase + p;
                const int lp = kps.level[rs];
                before = lp < level || (lp == level && (int)kps.y[rs] / c < cy_lo);
            }
            const int cnt = __popcll((__ballot(before) >> gshift) & 0xFFFFull);
            if (cnt == 0) {
                hi = lo;
            } else {
                const int pt = lo + (cnt - 1) * step;
                hi = min(pt + step, hi);
                lo = pt + 1;
            }
        }
        start = lo;
        end = nr;
    } else {
        // (clamped to [0, nr]: with keypoints out of canonical order some
        // entries are not written, and no read may leave the image's slots)
        start = min(max(tab[rl.row_tab + cy_lo], 0), nr);
        end = min(max(tab[rl.row_tab + cy_hi + 1], start), nr);
    }

    // key = distance << 40 | |dy| << 32 | disparity << 16 | index (no candidate: all ones)
    uint64_t key = ~(uint64_t)0;
    for (int j = start + k; j < end; j += ST_GROUP) {
        const int64_t rs = rbase + j;
        if constexpr (SEARCH) {
            if (kps.level[rs] != level || (int)kps.y[rs] / c > cy_hi) break;   // past the last candidate row
        }
        int dy = (int)kps.y[rs] - y;
        dy = dy < 0 ? -dy : dy;
        if (dy > a.band) continue;
        const int dd = x0 - (int)kps.x0[rs];
        if (dd < 0 || dd > a.d_max) continue;
        uint32_t h = 0;
#pragma unroll
        for (int w = 0; w < 8; w++) h += __popc(d[w] ^ desc[rs * 8 + w]);
        const uint64_t kj = ((uint64_t)h << 40) | ((uint64_t)dy << 32) | ((uint64_t)dd << 16) | (uint64_t)j;
        key = kj < key ? kj : key;
    }
#pragma unroll
    for (int m = ST_GROUP / 2; m > 0; m >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)key, m, ST_GROUP);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(key >> 32), m, ST_GROUP);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        key = o < key ? o : key;
    }
    if (k != 0) return;
    const int64_t o = (int64_t)pair * a.n_max + i;
    const uint32_t bd = (uint32_t)(key >> 40);
    if (key != ~(uint64_t)0 && (int)bd <= a.match_th) {
        midx[o] = (int32_t)(key & 0xFFFFu);
        mdist[o] = (uint16_t)bd;
        mdisp[o] = (int16_t)((key >> 16) & 0xFFFFu);
    } else {
        midx[o] = -1;
        mdist[o] = 0xFFFF;
        mdisp[o] = -1;
    }
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t stereo_match(const vsfe_ctx *ctx, const vsfe_batch *b, const vsfe_kp_soa *kps,
                                const int32_t *kp_count, const uint32_t *desc, int32_t *match_idx,
                                uint16_t *match_dist, int16_t *match_disp, int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!kps || !kp_count || !desc || !match_idx || !match_dist || !match_disp) return fail(VSFE_EINVAL, "null buffer");
    if (!kps->y || !kps->level || !kps->x0) return fail(VSFE_EINVAL, "null keypoint array");
    if (!b->pairs_ok) return fail(VSFE_EINVAL, "stereo_match needs pairs of equal-size images (2i, 2i+1)");
    StereoArgs a;
    for (int l = 0; l < VSFE_MAX_LEVELS; l++) a.cell[l] = ctx->cell[l] > 0 ? ctx->cell[l] : 1;
    a.n_max = ctx->p.n_max;
    a.n_pairs = b->n_images / 2;
    a.d_max = ctx->p.d_max;
    a.match_th = ctx->p.match_th;
    a.band = ctx->p.row_band;
    const int64_t n = (int64_t)a.n_pairs * a.n_max;
    if (n <= 0) return VSFE_OK;
    if (!b->d_row_tab) return fail(VSFE_EINVAL, "batch has no row-start table");
    if (n >= ((int64_t)1 << 27)) return fail(VSFE_ECAPACITY, "too many keypoint slots");
    const hipStream_t st = (hipStream_t)stream;
    if (n < 16384) {
        // small batches: the candidate rows are searched for, no table launch
        hipLaunchKernelGGL((stereo_kernel<16, true>), dim3((unsigned)((n * 16 + 255) / 256)), dim3(256), 0, st,
                           b->d_images, *kps, kp_count, desc, match_idx, match_dist, match_disp, b->d_row_tab, a);
        return check_launch("stereo_match");
    }
    const int64_t nt = (int64_t)a.n_pairs * (a.n_max + 1);
    hipLaunchKernelGGL(row_table_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, b->d_images, *kps,
                       kp_count, b->d_row_tab, a);
    rc = check_launch("stereo_match (row table)");
    if (rc) return rc;
    if (n < 131072)
        hipLaunchKernelGGL((stereo_kernel<4, false>), dim3((unsigned)((n * 4 + 255) / 256)), dim3(256), 0, st,
                           b->d_images, *kps, kp_count, desc, match_idx, match_dist, match_disp, b->d_row_tab, a);
    else
        hipLaunchKernelGGL((stereo_kernel<1, false>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           b->d_images, *kps, kp_count, desc, match_idx, match_dist, match_disp, b->d_row_tab, a);
    return check_launch("stereo_match");
}
