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
// allocation, no memset); then one thread per query visits only the cells
// its window overlaps.  The order inside a bucket depends on atomics, but
// the result does not: ties are broken by the reference index.
#include "vsfe_internal.h"

namespace vsfe {

struct MatchArgs {
    int n_max, n_images, radius, level_band, match_th, ratio_pct;
};

// workspace: counts | cursor | start (n_cells0 each) | list (kp_capacity)
struct MatchWs {
    int32_t *counts, *cursor, *start, *list;
};

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
                                                         const int32_t *__restrict__ ref_count, MatchWs ws,
                                                         MatchArgs a) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int img = (int)(s / a.n_max), j = (int)(s - (int64_t)img * a.n_max);
    if (img >= a.n_images || j >= ref_count[img]) return;
    const ImageDev &im = imgs[img];
    const int64_t slot = im.kp_offset + j;
    const int pos = atomicAdd(&ws.cursor[bucket_of(im, ref.x0[slot], ref.y0[slot])], 1);
    ws.list[im.kp_offset + pos] = j;
}

__global__ __launch_bounds__(256) void fm_match_kernel(const ImageDev *__restrict__ imgs, vsfe_kp_soa q,
                                                       const int32_t *__restrict__ q_count,
                                                       const uint32_t *__restrict__ q_desc, vsfe_kp_soa ref,
                                                       const uint32_t *__restrict__ ref_desc, MatchWs ws, MatchArgs a,
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
    for (int cy = ay0; cy <= ay1; cy++)
        for (int cx = ax0; cx <= ax1; cx++) {
            const int64_t cell = im.cell0_offset + (int64_t)cy * l0.ncx + cx;
            const int b0 = ws.start[cell], n = ws.counts[cell];
            for (int k = 0; k < n; k++) {
                const int j = ws.list[im.kp_offset + b0 + k];
                const int64_t rs = im.kp_offset + j;
                const int dx = x0 - (int)ref.x0[rs], dy = y0 - (int)ref.y0[rs], dl = lq - (int)ref.level[rs];
                if (dx < -r || dx > r || dy < -r || dy > r || dl < -a.level_band || dl > a.level_band) continue;
                int h = 0;
#pragma unroll
                for (int w = 0; w < 8; w++) h += __popc(d[w] ^ ref_desc[rs * 8 + w]);
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
    *bytes = (3 * b->info.n_cells0 + b->info.kp_capacity) * (int64_t)sizeof(int32_t);
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
    int32_t *w32 = (int32_t *)workspace;
    MatchWs ws{w32, w32 + n0, w32 + 2 * n0, w32 + 3 * n0};
    hipStream_t st = (hipStream_t)stream;
    const unsigned blocks = (unsigned)((slots + 255) / 256);
    hipLaunchKernelGGL(fm_clear_kernel, dim3((unsigned)std::min<int64_t>((n0 + 255) / 256, 4096)), dim3(256), 0, st,
                       ws.counts, n0);
    hipLaunchKernelGGL(fm_count_kernel, dim3(blocks), dim3(256), 0, st, b->d_images, *ref, ref_count, ws, a);
    hipLaunchKernelGGL(fm_scan_kernel, dim3(b->n_images), dim3(1024), 0, st, b->d_images, ws);
    hipLaunchKernelGGL(fm_scatter_kernel, dim3(blocks), dim3(256), 0, st, b->d_images, *ref, ref_count, ws, a);
    hipLaunchKernelGGL(fm_match_kernel, dim3(blocks), dim3(256), 0, st, b->d_images, *query, query_count, query_desc,
                       *ref, ref_desc, ws, a, match_idx, dist1, dist2);
    return check_launch("feature_match");
}
