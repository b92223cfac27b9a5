// Descriptor matching of a frame's keypoints against reference keypoints --
// the previous frame's, or map points projected into the frame (the
// middle-end's "Descriptor Matching" beside "Conic Projections", Sec. III-3,
// Fig. "slampipeline").
//
// Reference j is a candidate of query i when their native-scale positions
// differ by at most `radius` in x and y and their levels by at most
// `level_band`; best = least Hamming distance (ties: smaller index),
// second = least distance among the other candidates; accepted when
// best <= match_th and, with ratio_pct > 0 and a second candidate,
// 100 best < ratio_pct second.
//
// GPU mapping: the references of every image are bucketed by native-scale
// cell (the level-0 cell grid) with a counting sort in the caller's
// workspace (count, per-image scan, scatter: four small launches, no
// allocation, no memset).  The scatter writes each reference's packed
// position, level and index (8 bytes) and its descriptor (32 bytes) in
// bucket order, so the cells of one cell row of a query's window are one
// contiguous run whose descriptors load without waiting for the position
// check.  One thread per query walks the runs of the cell rows its window
// overlaps.  The order inside a bucket depends on atomics, but the result
// does not: ties are broken by the reference index.
#include "vsfe_internal.h"

namespace vsfe {

struct MatchArgs {
    int n_max, n_images, radius, level_band, match_th, ratio_pct;
};

// workspace: counts | cursor | start (n_cells0 each) | entry (kp_capacity)
// | desc (kp_capacity x 32 bytes), each section 256-byte aligned.  entry =
// (x0 | y0 << 16, index | level << 16): x0, y0 < 2^13, index < 2^16.
struct MatchWs {
    int32_t *counts, *cursor, *start;
    int2 *entry;
    uint4 *desc;
};

__host__ __device__ constexpr int64_t fm_align(int64_t n) { return (n + 255) & ~(int64_t)255; }

__global__ void fm_clear_kernel(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// native-scale cell of a position (positions past the grid go to its edge cells)
__device__ __forceinline__ int64_t bucket_of(const ImageDev &im, int x0, int y0) {
    const LevelDev &l0 = im.lv[0];
    const int cx = min(x0 / l0.cell, l0.ncx - 1), cy = min(y0 / l0.cell, l0.ncy - 1);
    return im.cell0_offset + (int64_t)cy * l0.ncx + cx;
}

__global__ __launch_bounds__(256) void fm_count_kernel(const ImageDev *__restrict__ imgs, vsfe_kp_soa ref,
                                                       const int32_t *__restrict__ ref_count, MatchWs ws, MatchArgs a) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int img = (int)(s / a.n_max), j = (int)(s - (int64_t)img * a.n_max);
    if (img >= a.n_images || j >= ref_count[img]) return;
    const ImageDev &im = imgs[img];
    const int64_t slot = im.kp_offset + j;
    atomicAdd(&ws.counts[bucket_of(im, ref.x0[slot], ref.y0[slot])], 1);
}

// Exclusive prefix sum of one image's bucket counts (one block per image):
// start[c] and cursor[c] = number of references in the image's earlier cells.
__global__ __launch_bounds__(1024) void fm_scan_kernel(const ImageDev *__restrict__ imgs, MatchWs ws) {
    __shared__ int32_t s_wave[16];
    __shared__ int32_t s_carry;
    const ImageDev &im = imgs[blockIdx.x];
    const int64_t c0 = im.cell0_offset;
    const int n = im.lv[0].ncx * im.lv[0].ncy;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int i = base + tid;
        const int v = i < n ? ws.counts[c0 + i] : 0;
        int incl = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(incl, d);
            if (lane >= d) incl += u;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        int before = s_carry;
        for (int w = 0; w < wave; w++) before += s_wave[w];
        if (i < n) {
            ws.start[c0 + i] = before + incl - v;
            ws.cursor[c0 + i] = before + incl - v;
        }
        __syncthreads();
        if (tid == 1023) s_carry = before + incl;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void fm_scatter_kernel(const ImageDev *__restrict__ imgs, vsfe_kp_soa ref,
                                                         const int32_t *__restrict__ ref_count,
                                                         const uint32_t *__restrict__ ref_desc, MatchWs ws,
                                                         MatchArgs a) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int img = (int)(s / a.n_max), j = (int)(s - (int64_t)img * a.n_max);
    if (img >= a.n_images || j >= ref_count[img]) return;
    const ImageDev &im = imgs[img];
    const int64_t slot = im.kp_offset + j;
    const int x0 = ref.x0[slot], y0 = ref.y0[slot];
    const int pos = atomicAdd(&ws.cursor[bucket_of(im, x0, y0)], 1);
    const int64_t o = im.kp_offset + pos;
    ws.entry[o] = make_int2(x0 | (y0 << 16), j | ((int)ref.level[slot] << 16));
    const uint32_t *dsrc = ref_desc + slot * 8;
    ws.desc[2 * o] = make_uint4(dsrc[0], dsrc[1], dsrc[2], dsrc[3]);
    ws.desc[2 * o + 1] = make_uint4(dsrc[4], dsrc[5], dsrc[6], dsrc[7]);
}

__global__ __launch_bounds__(256) void fm_match_kernel(const ImageDev *__restrict__ imgs, vsfe_kp_soa q,
                                                       const int32_t *__restrict__ q_count,
                                                       const uint32_t *__restrict__ q_desc, MatchWs ws, MatchArgs a,
                                                       int32_t *__restrict__ midx, uint16_t *__restrict__ d1,
                                                       uint16_t *__restrict__ d2) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int img = (int)(s / a.n_max), i = (int)(s - (int64_t)img * a.n_max);
    if (img >= a.n_images || i >= q_count[img]) return;
    const ImageDev &im = imgs[img];
    const LevelDev &l0 = im.lv[0];
    const int64_t qs = im.kp_offset + i;
    const int x0 = q.x0[qs], y0 = q.y0[qs], lq = q.level[qs];
    uint32_t d[8];
#pragma unroll
    for (int w = 0; w < 8; w++) d[w] = q_desc[qs * 8 + w];
    const int r = a.radius, c = l0.cell;
    const int ax0 = max(x0 - r, 0) / c, ax1 = min((x0 + r) / c, l0.ncx - 1);
    const int ay0 = max(y0 - r, 0) / c, ay1 = min((y0 + r) / c, l0.ncy - 1);
    int best = -1, bd = 0, sd = -1;
    for (int cy = ay0; cy <= ay1; cy++) {
        // cells ax0..ax1 of this row are consecutive buckets: one run
        const int64_t row = im.cell0_offset + (int64_t)cy * l0.ncx;
        const int b0 = ws.start[row + ax0], b1 = ws.start[row + ax1] + ws.counts[row + ax1];
        for (int p = b0; p < b1; p++) {
            const int64_t o = im.kp_offset + p;
            const int2 e = ws.entry[o];
            const uint4 da = ws.desc[2 * o], db = ws.desc[2 * o + 1];
            const int dx = x0 - (e.x & 0xFFFF), dy = y0 - (e.x >> 16), dl = lq - (e.y >> 16);
            if (dx < -r || dx > r || dy < -r || dy > r || dl < -a.level_band || dl > a.level_band) continue;
            const int j = e.y & 0xFFFF;
            const int h = __popc(d[0] ^ da.x) + __popc(d[1] ^ da.y) + __popc(d[2] ^ da.z) + __popc(d[3] ^ da.w) +
                          __popc(d[4] ^ db.x) + __popc(d[5] ^ db.y) + __popc(d[6] ^ db.z) + __popc(d[7] ^ db.w);
            // (best, runner-up) in any visiting order: the least distance,
            // ties to the smaller index; the runner-up is the least of the rest
            if (best < 0 || h < bd || (h == bd && j < best)) {
                if (best >= 0) sd = sd < 0 ? bd : min(sd, bd);
                best = j;
                bd = h;
            } else {
                sd = sd < 0 ? h : min(sd, h);
            }
        }
    }
    bool ok = best >= 0 && bd <= a.match_th;
    if (ok && a.ratio_pct > 0 && sd >= 0) ok = 100 * bd < a.ratio_pct * sd;
    midx[qs] = ok ? best : -1;
    d1[qs] = best >= 0 ? (uint16_t)bd : (uint16_t)0xFFFF;
    d2[qs] = sd >= 0 ? (uint16_t)sd : (uint16_t)0xFFFF;
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t vsfe_feature_match_workspace(const vsfe_batch *b, int64_t *bytes) {
    if (!b || !bytes) return fail(VSFE_EINVAL, "null argument");
    const int64_t cap = b->info.kp_capacity;
    *bytes = fm_align(3 * b->info.n_cells0 * (int64_t)sizeof(int32_t)) + fm_align(cap * 8) + cap * 32;
    return VSFE_OK;
}

extern "C" int32_t feature_match(const vsfe_ctx *ctx, const vsfe_batch *b, const vsfe_kp_soa *query,
                                 const int32_t *query_count, const uint32_t *query_desc, const vsfe_kp_soa *ref,
                                 const int32_t *ref_count, const uint32_t *ref_desc, int32_t radius, int32_t level_band,
                                 int32_t match_th, int32_t ratio_pct, void *workspace, int32_t *match_idx,
                                 uint16_t *dist1, uint16_t *dist2, int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!query || !query_count || !query_desc || !ref || !ref_count || !ref_desc || !workspace || !match_idx ||
        !dist1 || !dist2)
        return fail(VSFE_EINVAL, "null buffer");
    if (!query->x0 || !query->y0 || !query->level || !ref->x0 || !ref->y0 || !ref->level)
        return fail(VSFE_EINVAL, "null keypoint array");
    if (radius < 0 || radius > 255) return fail(VSFE_EINVAL, "radius out of 0..255");
    if (level_band < 0 || level_band >= VSFE_MAX_LEVELS) return fail(VSFE_EINVAL, "level_band out of 0..11");
    if (match_th < 0 || match_th > 256) return fail(VSFE_EINVAL, "match_th out of 0..256");
    if (ratio_pct < 0 || ratio_pct > 100) return fail(VSFE_EINVAL, "ratio_pct out of 0..100");
    MatchArgs a;
    a.n_max = ctx->p.n_max;
    a.n_images = b->n_images;
    a.radius = radius;
    a.level_band = level_band;
    a.match_th = match_th;
    a.ratio_pct = ratio_pct;
    const int64_t n0 = b->info.n_cells0, slots = b->info.kp_capacity;
    if (slots <= 0 || n0 <= 0) return VSFE_OK;
    if (slots >= ((int64_t)1 << 31)) return fail(VSFE_ECAPACITY, "more than 2^31 keypoint slots");
    if ((uintptr_t)workspace & 15) return fail(VSFE_EINVAL, "workspace not 16-byte aligned");
    int32_t *w32 = (int32_t *)workspace;
    uint8_t *w8 = (uint8_t *)workspace;
    const int64_t e_at = fm_align(3 * n0 * (int64_t)sizeof(int32_t)), d_at = e_at + fm_align(slots * 8);
    MatchWs ws{w32, w32 + n0, w32 + 2 * n0, (int2 *)(w8 + e_at), (uint4 *)(w8 + d_at)};
    hipStream_t st = (hipStream_t)stream;
    const unsigned blocks = (unsigned)((slots + 255) / 256);
    hipLaunchKernelGGL(fm_clear_kernel, dim3((unsigned)std::min<int64_t>((n0 + 255) / 256, 4096)), dim3(256), 0, st,
                       ws.counts, n0);
    hipLaunchKernelGGL(fm_count_kernel, dim3(blocks), dim3(256), 0, st, b->d_images, *ref, ref_count, ws, a);
    hipLaunchKernelGGL(fm_scan_kernel, dim3(b->n_images), dim3(1024), 0, st, b->d_images, ws);
    hipLaunchKernelGGL(fm_scatter_kernel, dim3(blocks), dim3(256), 0, st, b->d_images, *ref, ref_count, ref_desc, ws,
                       a);
    hipLaunchKernelGGL(fm_match_kernel, dim3(blocks), dim3(256), 0, st, b->d_images, *query, query_count, query_desc,
                       ws, a, match_idx, dist1, dist2);
    return check_launch("feature_match");
}
