// ORB orientation and rBRIEF descriptors for all levels in one launch
// (Sec. III-2: Gaussian smoothing, then extraction for every scale at once).
//
// One 64-lane wave per keypoint.  The wave stages the 37 x 37 neighbourhood
// of its keypoint in LDS (coordinates clamped to the level, which makes the
// clamp-to-edge smoothing exact), then
//   * intensity centroid m10 = sum u I, m01 = sum v I over u^2 + v^2 <= 225
//     on the unsmoothed level, reduced across the wave;
//   * orientation bin: 30 lanes compare m with the Q14 bin boundaries at
//     6 + 12 j degrees by exact integer half-plane / cross-product tests,
//     a ballot counts them (bin = count mod 30, 0 for m = 0);
//   * smoothing only of the 31 x 31 patch the tests can touch, separable
//     7-tap [18 33 49 56 49 33 18] / 256, each pass rounded half up;
//   * 256 tests on the bin-rotated pattern (precomputed per bin in the
//     context), 64 per ballot, written as 8 words.
// The whole-level blurred pyramid never touches HBM.
#include "vsfe_internal.h"

namespace vsfe {

constexpr int ORB_R = 37, ORB_P = 31;
constexpr int ORB_WAVES = 4;

struct OrbArgs {
    OrbTables tab;
    int n_max, n_images, blur;
};

__device__ __forceinline__ int half_plane(int64_t x, int64_t y) { return (y < 0 || (y == 0 && x < 0)) ? 1 : 0; }

__global__ __launch_bounds__(256) void orb_kernel(const ImageDev *__restrict__ imgs, const uint8_t *__restrict__ images,
                                                  const uint8_t *__restrict__ pyr, vsfe_kp_soa kps,
                                                  const int32_t *__restrict__ kp_count,
                                                  const int8_t *__restrict__ pat_rot, uint32_t *__restrict__ desc,
                                                  OrbArgs a) {
    __shared__ uint8_t s_raw[ORB_WAVES][ORB_R * ORB_R + 7];
    __shared__ uint8_t s_h[ORB_WAVES][ORB_R * ORB_P + 5];
    __shared__ uint8_t s_b[ORB_WAVES][ORB_P * ORB_P + 3];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t slot = (int64_t)blockIdx.x * ORB_WAVES + wave;
    const int image = (int)(slot / a.n_max);
    const int i = (int)(slot - (int64_t)image * a.n_max);
    const bool active = image < a.n_images && i < kp_count[image];

    int x = 0, y = 0, lvl = 0;
    LevelDev lv{};
    if (active) {
        x = kps.x[slot];
        y = kps.y[slot];
        lvl = kps.level[slot];
        lv = imgs[image].lv[lvl];
        const uint8_t *src = (lvl == 0 ? images : pyr) + lv.offset;
        for (int q = lane; q < ORB_R * ORB_R; q += 64) {
            const int r = q / ORB_R, cc = q - r * ORB_R;
            const int gy = min(max(y - 18 + r, 0), lv.h - 1);
            const int gx = min(max(x - 18 + cc, 0), lv.w - 1);
            s_raw[wave][q] = src[(int64_t)gy * lv.pitch + gx];
        }
    }
    __syncthreads();
    int m10 = 0, m01 = 0;
    if (active) {
        for (int q = lane; q < ORB_P * ORB_P; q += 64) {
            const int v = q / ORB_P - 15, u = q % ORB_P - 15;
            if (u * u + v * v <= 225) {
                const int I = s_raw[wave][(18 + v) * ORB_R + 18 + u];
                m10 += u * I;
                m01 += v * I;
            }
        }
        if (a.blur) {
            for (int q = lane; q < ORB_R * ORB_P; q += 64) {
                const int r = q / ORB_P, cc = q - r * ORB_P;
                const uint8_t *p = &s_raw[wave][r * ORB_R + cc];
                const int s = 18 * (p[0] + p[6]) + 33 * (p[1] + p[5]) + 49 * (p[2] + p[4]) + 56 * p[3];
                s_h[wave][q] = (uint8_t)((s + 128) >> 8);
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m10 += __shfl_xor(m10, o);
        m01 += __shfl_xor(m01, o);
    }
    __syncthreads();
    if (active) {
        for (int q = lane; q < ORB_P * ORB_P; q += 64) {
            const int r = q / ORB_P, cc = q - r * ORB_P;
            if (a.blur) {
                const uint8_t *p = &s_h[wave][r * ORB_P + cc];
                const int s = 18 * (p[0] + p[6 * ORB_P]) + 33 * (p[ORB_P] + p[5 * ORB_P]) +
                              49 * (p[2 * ORB_P] + p[4 * ORB_P]) + 56 * p[3 * ORB_P];
                s_b[wave][q] = (uint8_t)((s + 128) >> 8);
            } else {
                s_b[wave][q] = s_raw[wave][(r + 3) * ORB_R + cc + 3];
            }
        }
    }
    // orientation bin: lane j < 30 tests angle(m) >= angle(boundary j)
    bool ge = false;
    if (lane < 30) {
        const int64_t bx = a.tab.bin_x[lane], by = a.tab.bin_y[lane];
        const int hm = half_plane(m10, m01), hb = half_plane(bx, by);
        ge = hm != hb ? hm > hb : (bx * (int64_t)m01 - by * (int64_t)m10 >= 0);
    }
    const uint64_t gem = __ballot(ge);
    int bin = (m10 == 0 && m01 == 0) ? 0 : (__popcll(gem) % 30);
    __syncthreads();
    if (active) {
        const int8_t *pr = pat_rot + (int64_t)bin * 256 * 4;
        uint32_t words[8];
#pragma unroll
        for (int rnd = 0; rnd < 4; rnd++) {
            const int t = rnd * 64 + lane;
            const char4 q = *(const char4 *)(pr + 4 * t);
            const int va = s_b[wave][(15 + q.y) * ORB_P + 15 + q.x];
            const int vb = s_b[wave][(15 + q.w) * ORB_P + 15 + q.z];
            const uint64_t bits = __ballot(va < vb);
            words[2 * rnd] = (uint32_t)bits;
            words[2 * rnd + 1] = (uint32_t)(bits >> 32);
        }
        if (lane < 8) {
            uint32_t w = words[0];
#pragma unroll
            for (int k = 1; k < 8; k++)
                if (lane == k) w = words[k];
            desc[slot * 8 + lane] = w;
        }
        if (lane == 0) kps.bin[slot] = (uint8_t)bin;
    }
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t orb_describe(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images, const uint8_t *pyr,
                                const vsfe_kp_soa *kps, const int32_t *kp_count, uint32_t *desc, int32_t *status,
                                void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !kps || !kp_count || !desc || (!pyr && b->info.n_levels > 1)) return fail(VSFE_EINVAL, "null buffer");
    if (!kps->x || !kps->y || !kps->level || !kps->bin) return fail(VSFE_EINVAL, "null keypoint array");
    if (ctx->p.border < 15) return fail(VSFE_EINVAL, "orb_describe needs border >= 15");
    OrbArgs a;
    a.tab = ctx->tables;
    a.n_max = ctx->p.n_max;
    a.n_images = b->n_images;
    a.blur = ctx->p.blur;
    const int64_t slots = b->info.kp_capacity;
    const int64_t blocks = (slots + ORB_WAVES - 1) / ORB_WAVES;
    if (blocks <= 0) return VSFE_OK;
    hipLaunchKernelGGL(orb_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, b->d_images, images, pyr,
                       *kps, kp_count, ctx->d_pattern_rot, desc, a);
    return check_launch("orb_describe");
}
