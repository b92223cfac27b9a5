// Learned cell proposer: a small CNN on pyramid level 3 that predicts which
// native-scale cells will hold final keypoints, so the exact detector runs
// only there (the gating itself is in fast_br_detect).
//
// Network (one logit per stride-8 position of level 3):
//   x = (I_3 - 128) / 128 -> conv3x3 s2 (1 -> 16) -> ReLU -> conv3x3 s2
//   (16 -> 32) -> ReLU -> conv3x3 s2 (32 -> 32) -> ReLU -> conv1x1 (32 -> 1).
// Padding 1, ceil(in / 2) outputs per axis.  Parameters are one flat
// vector, OIHW weights followed by biases per layer.  Weights and stored
// activations are bfloat16 (NHWC), sums are float32.
//
//  * conv1 (K = 9 taps, padded to 16) runs on v_mfma_f32_16x16x16_bf16;
//  * conv2 (K = 144) and conv3 (K = 288) are implicit GEMMs on
//    v_mfma_f32_16x16x32_bf16: one wave computes 32 channels x 16 output
//    pixels, each lane feeding 8 consecutive channels of one tap as its
//    K slice (weights repacked to [co][tap][ci]); the 1x1 head is fused in
//    conv3's epilogue with a shuffle reduction over the channel groups;
//  * inference (cnn_propose) runs the three layers and the head fused in
//    one kernel per 4 x 8 tile of grid positions, activations in LDS; the
//    layer-by-layer kernels (cnn_forward) keep the activations for training;
//  * cell logits: per native-scale cell, the maximum over the grid
//    positions whose projected centre ((8 j + 4) S_3 + 2^15) >> 16 falls in
//    it (a cell with none is always kept);
//  * training: mean binary cross-entropy with a positive-class weight,
//    backward in float32 on the VALU, weight gradients as per-block partial
//    sums reduced in a fixed order (deterministic), then Adam.
#include <string.h>

#include <algorithm>

#include "vsfe_internal.h"

namespace vsfe {

constexpr int CNN_NPARAM = 14081;
constexpr int P_W1 = 0, P_B1 = 144, P_W2 = 160, P_B2 = 4768, P_W3 = 4800, P_B3 = 14016, P_W4 = 14048, P_B4 = 14080;
constexpr int CNN_PARTS = 256;            // partial-sum blocks of the weight gradients

struct CnnImg {
    int32_t w0, h0, w3, h3, w1, h1, w2, h2, w4, h4, ncx0, ncy0, cell0, pitch3;
    int64_t lvl3;                      // byte offset of level 3 in the pyramid buffer
    int64_t px1, px2, px4;             // first pixel of this image in each layer's arrays
    int64_t c0;                        // first native-scale cell
};

struct CnnPlan {
    int n = 0;
    std::vector<CnnImg> h_img;
    CnnImg *d_img = nullptr;
    // prefixes (n + 1 each): px1, px2, px4, tiles2, tiles4, cells, tiles1, fused tiles
    std::vector<int32_t> h_pre;
    int32_t *d_pre = nullptr;
    int64_t px1 = 0, px2 = 0, px4 = 0, t2 = 0, t4 = 0, cells = 0, t1 = 0, tf = 0;
    int64_t off_wp2 = 0, off_wp3 = 0, off_a1 = 0, off_a2 = 0, off_a3 = 0, off_g1 = 0, off_g2 = 0, off_g3 = 0,
            off_dz = 0, off_lz = 0, off_part = 0, total = 0;
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf(uint16_t v) { return __builtin_bit_cast(float, (uint32_t)v << 16); }
__device__ __forceinline__ uint16_t to_bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// largest i with pre[i] <= g (pre is nondecreasing, pre[0] = 0)
__device__ __forceinline__ int find_image(const int32_t *pre, int n, int64_t g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// --------------------------------------------------------------- forward
// Repack conv2 / conv3 weights from OIHW to [co][tap][ci] (bf16).
__global__ void cnn_pack_kernel(const uint16_t *__restrict__ prm, uint16_t *__restrict__ wp2, uint16_t *__restrict__ wp3) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 32 * 9 * 16) {
        const int co = i / (9 * 16), t = (i / 16) % 9, ci = i % 16;
        wp2[i] = prm[P_W2 + (co * 16 + ci) * 9 + t];
    }
    if (i < 32 * 9 * 32) {
        const int co = i / (9 * 32), t = (i / 32) % 9, ci = i % 32;
        wp3[i] = prm[P_W3 + (co * 32 + ci) * 9 + t];
    }
}

// All three convolutions run on MFMA with the weights as the A operand
// (row = output channel) and the activations as the B operand (column =
// output pixel), so each lane ends with 4 consecutive channels of one pixel
// and stores them as one 8-byte NHWC write.  Lane l: pixel l % 16, K slice
// (l / 16); accumulator r of lane l is channel 4 (l / 16) + r.  Both forward
// paths use the helpers below, so their activations and logits are
// bit-identical.
//
// conv1 (1 -> 16, K = 9 taps zero-padded to 16) on v_mfma_f32_16x16x16_bf16;
// the input x = (I - 128) / 128 is exact in bfloat16.
typedef short i16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t x_bf(int v) { return to_bf((float)(v - 128) * (1.0f / 128.0f)); }

// A operand of conv1: w1[c][k] for channel c = lane % 16 and the lane's 4 taps
__device__ __forceinline__ i16x4 conv1_weights(const uint16_t *prm, int lane) {
    const int c = lane & 15, k0 = 4 * (lane >> 4);
    i16x4 w;
#pragma unroll
    for (int j = 0; j < 4; j++) w[j] = (short)(k0 + j < 9 ? prm[P_W1 + c * 9 + k0 + j] : 0);
    return w;
}

__device__ __forceinline__ f32x4 conv1_mfma(i16x4 w, i16x4 x) {
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w, x, zero, 0, 0, 0);
}

// bias + ReLU + bfloat16 of 4 consecutive channels, packed for one 8-byte store
__device__ __forceinline__ uint2 relu_pack4(f32x4 acc, const float *bias) {
    uint16_t v[4];
#pragma unroll
    for (int r = 0; r < 4; r++) v[r] = to_bf(fmaxf(acc[r] + bias[r], 0.0f));
    return make_uint2((uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16));
}

__device__ __forceinline__ float bf_lo(uint32_t v) { return bf((uint16_t)(v & 0xFFFFu)); }
__device__ __forceinline__ float bf_hi(uint32_t v) { return bf((uint16_t)(v >> 16)); }

// 1x1 head partial of one lane (its 8 channels), fixed order
__device__ __forceinline__ float head_part(uint2 p0, uint2 p1, const float *h0, const float *h1) {
    float s = 0.f;
    s += h0[0] * bf_lo(p0.x);
    s += h0[1] * bf_hi(p0.x);
    s += h0[2] * bf_lo(p0.y);
    s += h0[3] * bf_hi(p0.y);
    s += h1[0] * bf_lo(p1.x);
    s += h1[1] * bf_hi(p1.x);
    s += h1[2] * bf_lo(p1.y);
    s += h1[3] * bf_hi(p1.y);
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s;
}

// One wave: 16 consecutive conv1 pixels of one image (row-major), NHWC out.
__global__ __launch_bounds__(256) void cnn_conv1_kernel(const CnnImg *__restrict__ imgs,
                                                        const int32_t *__restrict__ pre_tiles, int n,
                                                        int64_t total_tiles, const uint8_t *__restrict__ pyr,
                                                        const uint16_t *__restrict__ prm, uint16_t *__restrict__ a1) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile >= total_tiles) return;
    const int i = find_image(pre_tiles, n, tile);
    const CnnImg im = imgs[i];
    const int npx = im.w1 * im.h1;
    const int m = lane & 15, grp = lane >> 4;
    const int pm = (int)(tile - pre_tiles[i]) * 16 + m;
    const int oy = pm / im.w1, ox = pm - oy * im.w1;
    i16x4 x;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int k = 4 * grp + j;
        const int iy = 2 * oy + k / 3 - 1, ix = 2 * ox + k % 3 - 1;
        const bool in = pm < npx && k < 9 && iy >= 0 && iy < im.h3 && ix >= 0 && ix < im.w3;
        x[j] = (short)(in ? x_bf(pyr[im.lvl3 + (int64_t)iy * im.pitch3 + ix]) : 0);
    }
    const f32x4 acc = conv1_mfma(conv1_weights(prm, lane), x);
    float bias[4];
#pragma unroll
    for (int r = 0; r < 4; r++) bias[r] = bf(prm[P_B1 + 4 * grp + r]);
    if (pm < npx) *(uint2 *)(a1 + (im.px1 + pm) * 16 + 4 * grp) = relu_pack4(acc, bias);
}

// Implicit-GEMM 3x3 stride-2 convolution CIN -> 32: K chunks of 32 (conv2:
// pairs of taps x 16 channels, the last padded; conv3: one tap x 32
// channels); A = packed weights [co][tap][ci], B = 8 channels of one tap of
// the lane's pixel.  Returns through acc0 (channels 0..15) and acc1 (16..31).
template <int CIN>
__device__ __forceinline__ void conv_weights(const uint16_t *wp, int lane, uint4 *w0, uint4 *w1) {
    constexpr int NCH = CIN == 16 ? 5 : 9;
    const int m = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int c = 0; c < NCH; c++) {
        const int t = CIN == 16 ? 2 * c + (grp >> 1) : c;
        const int ci0 = CIN == 16 ? 8 * (grp & 1) : 8 * grp;
        w0[c] = w1[c] = make_uint4(0, 0, 0, 0);
        if (t < 9) {
            w0[c] = *(const uint4 *)(wp + ((m * 9 + t) * CIN + ci0));
            w1[c] = *(const uint4 *)(wp + (((m + 16) * 9 + t) * CIN + ci0));
        }
    }
}

__device__ __forceinline__ void conv_mfma2(uint4 xv, uint4 w0, uint4 w1, f32x4 &acc0, f32x4 &acc1) {
    const bf16x8 x = __builtin_bit_cast(bf16x8, xv);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, w0), x, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, w1), x, acc1, 0, 0, 0);
}

template <int CIN, bool HEAD>
__global__ __launch_bounds__(256) void cnn_conv_mfma_kernel(const CnnImg *__restrict__ imgs,
                                                            const int32_t *__restrict__ pre_tiles, int n,
                                                            int64_t total_tiles, const uint16_t *__restrict__ ain,
                                                            uint16_t *__restrict__ aout, const uint16_t *__restrict__ wp,
                                                            const uint16_t *__restrict__ prm, float *__restrict__ z) {
    constexpr int NCH = CIN == 16 ? 5 : 9;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile >= total_tiles) return;
    const int i = find_image(pre_tiles, n, tile);
    const CnnImg im = imgs[i];
    const int in_w = CIN == 16 ? im.w1 : im.w2, in_h = CIN == 16 ? im.h1 : im.h2;
    const int out_w = CIN == 16 ? im.w2 : im.w4, out_h = CIN == 16 ? im.h2 : im.h4;
    const int64_t in_base = CIN == 16 ? im.px1 : im.px2, out_base = CIN == 16 ? im.px2 : im.px4;
    const int npx = out_w * out_h;
    const int m = lane & 15, grp = lane >> 4;
    const int pm = (int)(tile - pre_tiles[i]) * 16 + m;
    const bool valid = pm < npx;
    const int oy = valid ? pm / out_w : 0, ox = valid ? pm - oy * out_w : 0;
    uint4 w0[NCH], w1[NCH];
    conv_weights<CIN>(wp, lane, w0, w1);
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NCH; c++) {
        const int t = CIN == 16 ? 2 * c + (grp >> 1) : c;
        const int ci0 = CIN == 16 ? 8 * (grp & 1) : 8 * grp;
        uint4 xv = make_uint4(0, 0, 0, 0);
        if (t < 9) {
            const int iy = 2 * oy + t / 3 - 1, ix = 2 * ox + t % 3 - 1;
            if (valid && iy >= 0 && iy < in_h && ix >= 0 && ix < in_w)
                xv = *(const uint4 *)(ain + ((in_base + (int64_t)iy * in_w + ix) * CIN + ci0));
        }
        conv_mfma2(xv, w0[c], w1[c], acc0, acc1);
    }
    const int bias_at = CIN == 16 ? P_B2 : P_B3;
    float b0[4], b1[4];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        b0[r] = bf(prm[bias_at + 4 * grp + r]);
        b1[r] = bf(prm[bias_at + 16 + 4 * grp + r]);
    }
    const uint2 v0 = relu_pack4(acc0, b0), v1 = relu_pack4(acc1, b1);
    if (valid) {
        *(uint2 *)(aout + (out_base + pm) * 32 + 4 * grp) = v0;
        *(uint2 *)(aout + (out_base + pm) * 32 + 16 + 4 * grp) = v1;
    }
    if (HEAD) {
        float h0[4], h1[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            h0[r] = bf(prm[P_W4 + 4 * grp + r]);
            h1[r] = bf(prm[P_W4 + 16 + 4 * grp + r]);
        }
        const float part = head_part(v0, v1, h0, h1);
        if (grp == 0 && valid) z[out_base + pm] = part + bf(prm[P_B4]);
    }
}

// Fused inference forward: one 256-thread block computes a 4 x 8 tile of
// grid logits with every intermediate activation in LDS (level-3 input
// 39 x 71, conv1 19 x 35 x 16, conv2 9 x 17 x 32; positions outside an
// activation map are its zero padding).  Same helpers as the layer-by-layer
// kernels, so the logits are bit-identical to cnn_forward's.
constexpr int CF3H = 4, CF3W = 8;                         // grid positions per tile
constexpr int CF2H = 2 * CF3H + 1, CF2W = 2 * CF3W + 1;   // conv2 window  9 x 17
constexpr int CF1H = 2 * CF2H + 1, CF1W = 2 * CF2W + 1;   // conv1 window 19 x 35
constexpr int CF0H = 2 * CF1H + 1, CF0W = 2 * CF1W + 1;   // input window 39 x 71
constexpr int CF0S = CF0W + 1;                            // input row stride (u16)
constexpr int CF0D = (CF0W + 1 + 3) / 4;                  // dwords per input row (18)
constexpr int CF_LD = (CF0H * CF0D + 255) / 256;          // dword loads per thread (3)
constexpr int CF1N = CF1H * CF1W, CF2N = CF2H * CF2W;
constexpr int CF_U = CF2N * 32 > CF0H * CF0S ? CF2N * 32 : CF0H * CF0S;

__global__ __launch_bounds__(256) void cnn_fused_fwd_kernel(const CnnImg *__restrict__ imgs,
                                                            const int32_t *__restrict__ pre_tiles, int n,
                                                            const uint8_t *__restrict__ pyr,
                                                            const uint16_t *__restrict__ prm,
                                                            const uint16_t *__restrict__ wp2,
                                                            const uint16_t *__restrict__ wp3, float *__restrict__ z) {
    __shared__ __attribute__((aligned(16))) uint16_t s_a1[CF1N * 16];
    __shared__ __attribute__((aligned(16))) uint16_t s_u[CF_U];     // input, then conv2 output
    uint16_t *const s_c2 = s_u;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int m = lane & 15, grp = lane >> 4;
    const int bt = xcd_item(blockIdx.x, gridDim.x);
    const int i = find_image(pre_tiles, n, bt);
    const CnnImg im = imgs[i];
    const int lt = bt - pre_tiles[i];
    const int ntx = (im.w4 + CF3W - 1) / CF3W;
    const int Y3 = (lt / ntx) * CF3H, X3 = (lt % ntx) * CF3W;
    const int Y2 = 2 * Y3 - 1, X2 = 2 * X3 - 1, Y1 = 2 * Y2 - 1, X1 = 2 * X2 - 1, Y0 = 2 * Y1 - 1, X0 = 2 * X1 - 1;

    // A. level-3 input window as bfloat16.  X0 - 1 = 8 X3 - 8 is a multiple
    //    of 4 and rows start on 64-byte boundaries, so the window is read as
    //    aligned dwords (bytes past the level width are masked); all loads
    //    are issued before any is used.
    {
        uint32_t v[CF_LD];
#pragma unroll
        for (int k = 0; k < CF_LD; k++) {
            const int d = tid + 256 * k;
            const int rr = d / CF0D, j = d - rr * CF0D;
            const int gy = Y0 + rr, gx = X0 - 1 + 4 * j;
            const bool ok = d < CF0H * CF0D && gy >= 0 && gy < im.h3 && gx >= 0 && gx < im.w3;
            v[k] = ok ? *(const uint32_t *)(pyr + im.lvl3 + (int64_t)gy * im.pitch3 + gx) : 0u;
        }
#pragma unroll
        for (int k = 0; k < CF_LD; k++) {
            const int d = tid + 256 * k;
            if (d >= CF0H * CF0D) continue;
            const int rr = d / CF0D, j = d - rr * CF0D;
            const int gy = Y0 + rr, gx = X0 - 1 + 4 * j;
            const bool ok = gy >= 0 && gy < im.h3 && gx >= 0 && gx < im.w3;
#pragma unroll
            for (int bb = 0; bb < 4; bb++) {
                const int cc = 4 * j - 1 + bb;                  // window column of byte bb
                if (cc < 0 || cc >= CF0W) continue;
                s_u[rr * CF0S + cc] = ok && gx + bb < im.w3 ? x_bf((int)((v[k] >> (8 * bb)) & 255u)) : (uint16_t)0;
            }
        }
    }
    __syncthreads();

    // B. conv1: one pixel per lane and M tile, 4 channels per lane
    {
        const i16x4 w = conv1_weights(prm, lane);
        float bias[4];
#pragma unroll
        for (int r = 0; r < 4; r++) bias[r] = bf(prm[P_B1 + 4 * grp + r]);
        int toff[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int k = 4 * grp + j;
            toff[j] = k < 9 ? (k / 3) * CF0S + (k % 3) : -1;
        }
        const int vy0 = max(0, -Y1), vy1 = min(CF1H, im.h1 - Y1), vx0 = max(0, -X1), vx1 = min(CF1W, im.w1 - X1);
        for (int t = wave; t < (CF1N + 15) / 16; t += 4) {
            const int p = 16 * t + m;
            const int r1 = p / CF1W, c1 = p - r1 * CF1W;
            const int base = 2 * r1 * CF0S + 2 * c1;
            i16x4 x;
#pragma unroll
            for (int j = 0; j < 4; j++) x[j] = (short)(p < CF1N && toff[j] >= 0 ? s_u[base + toff[j]] : 0);
            const f32x4 acc = conv1_mfma(w, x);
            if (p < CF1N) {
                const bool in = r1 >= vy0 && r1 < vy1 && c1 >= vx0 && c1 < vx1;
                *(uint2 *)(s_a1 + p * 16 + 4 * grp) = in ? relu_pack4(acc, bias) : make_uint2(0, 0);
            }
        }
    }
    __syncthreads();

    // C. conv2 (16 -> 32)
    {
        uint4 w0[5], w1[5];
        conv_weights<16>(wp2, lane, w0, w1);
        float b0[4], b1[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            b0[r] = bf(prm[P_B2 + 4 * grp + r]);
            b1[r] = bf(prm[P_B2 + 16 + 4 * grp + r]);
        }
        const int vy0 = max(0, -Y2), vy1 = min(CF2H, im.h2 - Y2), vx0 = max(0, -X2), vx1 = min(CF2W, im.w2 - X2);
        for (int t2 = wave; t2 < (CF2N + 15) / 16; t2 += 4) {
            const int p = 16 * t2 + m;
            const bool valid = p < CF2N;
            const int r2 = valid ? p / CF2W : 0, c2 = valid ? p - r2 * CF2W : 0;
            f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 5; c++) {
                const int t = 2 * c + (grp >> 1), ci0 = 8 * (grp & 1);
                uint4 xv = make_uint4(0, 0, 0, 0);
                if (t < 9 && valid) xv = *(const uint4 *)(s_a1 + ((2 * r2 + t / 3) * CF1W + (2 * c2 + t % 3)) * 16 + ci0);
                conv_mfma2(xv, w0[c], w1[c], acc0, acc1);
            }
            if (valid) {
                const bool in = r2 >= vy0 && r2 < vy1 && c2 >= vx0 && c2 < vx1;
                *(uint2 *)(s_c2 + p * 32 + 4 * grp) = in ? relu_pack4(acc0, b0) : make_uint2(0, 0);
                *(uint2 *)(s_c2 + p * 32 + 16 + 4 * grp) = in ? relu_pack4(acc1, b1) : make_uint2(0, 0);
            }
        }
    }
    __syncthreads();

    // D. conv3 (32 -> 32) + 1x1 head: waves 0 and 1 take tile rows 2w, 2w + 1
    if (wave < CF3H / 2) {
        const int r3 = 2 * wave + (m >> 3), c3 = m & 7;
        uint4 w0[9], w1[9];
        conv_weights<32>(wp3, lane, w0, w1);
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; t++) {
            const uint4 xv = *(const uint4 *)(s_c2 + ((2 * r3 + t / 3) * CF2W + (2 * c3 + t % 3)) * 32 + 8 * grp);
            conv_mfma2(xv, w0[t], w1[t], acc0, acc1);
        }
        float b0[4], b1[4], h0[4], h1[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            b0[r] = bf(prm[P_B3 + 4 * grp + r]);
            b1[r] = bf(prm[P_B3 + 16 + 4 * grp + r]);
            h0[r] = bf(prm[P_W4 + 4 * grp + r]);
            h1[r] = bf(prm[P_W4 + 16 + 4 * grp + r]);
        }
        const float part = head_part(relu_pack4(acc0, b0), relu_pack4(acc1, b1), h0, h1);
        const int gy = Y3 + r3, gx = X3 + c3;
        if (grp == 0 && gy < im.h4 && gx < im.w4) z[im.px4 + (int64_t)gy * im.w4 + gx] = part + bf(prm[P_B4]);
    }
}

__global__ void cnn_cells_kernel(const CnnImg *__restrict__ imgs, const int32_t *__restrict__ pre_cells, int n,
                                 int64_t total, const float *__restrict__ z, float thresh,
                                 float *__restrict__ cell_logit, uint8_t *__restrict__ mask, int S3) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int i = find_image(pre_cells, n, g);
    const CnnImg im = imgs[i];
    const int c = (int)(g - im.c0);
    const int cy = c / im.ncx0, cx = c - cy * im.ncx0;
    auto proj = [&](int j, int lim) { return min((int)(((int64_t)(8 * j + 4) * S3 + 32768) >> 16), lim - 1); };
    // first grid column / row whose projected centre reaches the cell
    int j0 = max(0, (int)(((int64_t)cx * im.cell0 * 65536 / S3 - 4) / 8) - 2);
    while (j0 < im.w4 && proj(j0, im.w0) < cx * im.cell0) j0++;
    int i0 = max(0, (int)(((int64_t)cy * im.cell0 * 65536 / S3 - 4) / 8) - 2);
    while (i0 < im.h4 && proj(i0, im.h0) < cy * im.cell0) i0++;
    float best = -INFINITY;
    bool any = false;
    for (int a = i0; a < im.h4 && proj(a, im.h0) < (cy + 1) * im.cell0; a++)
        for (int b = j0; b < im.w4 && proj(b, im.w0) < (cx + 1) * im.cell0; b++) {
            best = fmaxf(best, z[im.px4 + (int64_t)a * im.w4 + b]);
            any = true;
        }
    if (!any) best = INFINITY;
    if (cell_logit) cell_logit[g] = best;
    if (mask) mask[g] = (uint8_t)(best >= thresh ? 1 : 0);
}

// --------------------------------------------------------------- backward
// dz = d(mean BCE)/dz, per-position loss, and the conv3 output gradient
// g3 = dz w4 [a3 > 0].
__global__ void cnn_head_bwd_kernel(int64_t total, const float *__restrict__ z, const float *__restrict__ target,
                                    float pos_weight, const uint16_t *__restrict__ prm,
                                    const uint16_t *__restrict__ a3, float *__restrict__ dz, float *__restrict__ lz,
                                    float *__restrict__ g3) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= total) return;
    const float zz = z[p], t = target[p];
    const float inv_n = 1.0f / (float)total;
    const float sp_pos = fmaxf(-zz, 0.f) + log1pf(expf(-fabsf(zz)));   // -log sigmoid(z)
    const float sp_neg = fmaxf(zz, 0.f) + log1pf(expf(-fabsf(zz)));    // -log(1 - sigmoid(z))
    const float s = 1.0f / (1.0f + expf(-zz));
    lz[p] = (pos_weight * t * sp_pos + (1.f - t) * sp_neg) * inv_n;
    const float d = (pos_weight * t * (s - 1.f) + (1.f - t) * s) * inv_n;
    dz[p] = d;
    for (int co = 0; co < 32; co++) {
        const float a = bf(a3[p * 32 + co]);
        g3[p * 32 + co] = a > 0.f ? d * bf(prm[P_W4 + co]) : 0.f;
    }
}

// Partial sums of the head gradients over a pixel range.
__global__ __launch_bounds__(256) void cnn_head_wgrad_kernel(int64_t total, const float *__restrict__ dz,
                                                             const uint16_t *__restrict__ a3,
                                                             float *__restrict__ part) {
    __shared__ float s_acc[256][33];
    const int64_t chunk = (total + CNN_PARTS - 1) / CNN_PARTS;
    const int64_t lo = blockIdx.x * chunk, hi = min(total, lo + chunk);
    float acc[33];
    for (int k = 0; k < 33; k++) acc[k] = 0.f;
    for (int64_t p = lo + threadIdx.x; p < hi; p += 256) {
        const float d = dz[p];
        for (int co = 0; co < 32; co++) acc[co] += d * bf(a3[p * 32 + co]);
        acc[32] += d;
    }
    for (int k = 0; k < 33; k++) s_acc[threadIdx.x][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < 33) {
        float s = 0.f;
        for (int t = 0; t < 256; t++) s += s_acc[t][threadIdx.x];
        part[(int64_t)blockIdx.x * CNN_NPARAM + (threadIdx.x < 32 ? P_W4 + threadIdx.x : P_B4)] = s;
    }
}

// Partial sums of a 3x3 stride-2 convolution's weight / bias gradients:
// dW[co][ci][t] = sum_p g[p][co] a[in(p, t)][ci].  U8IN: the input is the
// level-3 image, x = (I - 128) / 128.
template <int CIN, int COUT, bool U8IN>
__global__ __launch_bounds__(256) void cnn_wgrad_kernel(const CnnImg *__restrict__ imgs, const int32_t *__restrict__ pre_out,
                                                        int n, int64_t total, const float *__restrict__ g,
                                                        const uint16_t *__restrict__ ain, const uint8_t *__restrict__ pyr,
                                                        float *__restrict__ part, int w_at, int b_at) {
    constexpr int NW = COUT * 9 * CIN;
    constexpr int PER = NW < 256 * 9 ? (NW + 255) / 256 : 9;   // weights per thread (grid.y splits the rest)
    constexpr int PB = 16;                       // pixels staged per round
    const int wbase = blockIdx.y * 256 * PER;
    __shared__ float s_g[PB][COUT];
    __shared__ float s_a[PB][9 * CIN];
    const int64_t chunk = (total + CNN_PARTS - 1) / CNN_PARTS;
    const int64_t lo = blockIdx.x * chunk, hi = min(total, lo + chunk);
    float acc[PER], bacc = 0.f;
#pragma unroll
    for (int k = 0; k < PER; k++) acc[k] = 0.f;
    for (int64_t base = lo; base < hi; base += PB) {
        // stage the output gradients and input patches of PB pixels
        for (int q = threadIdx.x; q < PB * COUT; q += 256) {
            const int pp = q / COUT, co = q - pp * COUT;
            const int64_t p = base + pp;
            s_g[pp][co] = p < hi ? g[p * COUT + co] : 0.f;
        }
        for (int q = threadIdx.x; q < PB * 9 * CIN; q += 256) {
            const int pp = q / (9 * CIN), r = q - pp * 9 * CIN, t = r / CIN, ci = r - t * CIN;
            const int64_t p = base + pp;
            float v = 0.f;
            if (p < hi) {
                const int i = find_image(pre_out, n, p);
                const CnnImg im = imgs[i];
                const int ow = CIN == 1 ? im.w1 : (CIN == 16 ? im.w2 : im.w4);
                const int iw = CIN == 1 ? im.w3 : (CIN == 16 ? im.w1 : im.w2);
                const int ih = CIN == 1 ? im.h3 : (CIN == 16 ? im.h1 : im.h2);
                const int64_t ob = CIN == 1 ? im.px1 : (CIN == 16 ? im.px2 : im.px4);
                const int64_t ib = CIN == 16 ? im.px1 : im.px2;
                const int lp = (int)(p - ob), oy = lp / ow, ox = lp - oy * ow;
                const int iy = 2 * oy + t / 3 - 1, ix = 2 * ox + t % 3 - 1;
                if (iy >= 0 && iy < ih && ix >= 0 && ix < iw) {
                    if (U8IN) v = ((float)pyr[im.lvl3 + (int64_t)iy * im.pitch3 + ix] - 128.0f) * (1.0f / 128.0f);
                    else v = bf(ain[(ib + (int64_t)iy * iw + ix) * CIN + ci]);
                }
            }
            s_a[pp][r] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int w = wbase + threadIdx.x + 256 * k;
            if (w < NW) {
                const int co = w / (9 * CIN), r = w - co * 9 * CIN;
                float s = acc[k];
                for (int pp = 0; pp < PB; pp++) s += s_g[pp][co] * s_a[pp][r];
                acc[k] = s;
            }
        }
        if (blockIdx.y == 0 && threadIdx.x < COUT)
            for (int pp = 0; pp < PB; pp++) bacc += s_g[pp][threadIdx.x];
        __syncthreads();
    }
    float *out = part + (int64_t)blockIdx.x * CNN_NPARAM;
#pragma unroll
    for (int k = 0; k < PER; k++) {
        const int w = wbase + threadIdx.x + 256 * k;
        if (w < NW) {
            const int co = w / (9 * CIN), r = w - co * 9 * CIN, t = r / CIN, ci = r - t * CIN;
            out[w_at + (co * CIN + ci) * 9 + t] = acc[k];
        }
    }
    if (blockIdx.y == 0 && threadIdx.x < COUT) out[b_at + threadIdx.x] = bacc;
}

// Input gradient of a 3x3 stride-2 convolution (transposed-convolution
// gather), times the ReLU mask of the input activation.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void cnn_dgrad_kernel(const CnnImg *__restrict__ imgs, const int32_t *__restrict__ pre_in,
                                                        int n, int64_t total_in, const float *__restrict__ gout,
                                                        const uint16_t *__restrict__ ain, const uint16_t *__restrict__ prm,
                                                        int w_at, float *__restrict__ gin) {
    __shared__ float s_w[COUT * CIN * 9];
    for (int q = threadIdx.x; q < COUT * CIN * 9; q += 256) s_w[q] = bf(prm[w_at + q]);
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total_in * CIN) return;
    const int64_t q = e / CIN;
    const int ci = (int)(e - q * CIN);
    const int i = find_image(pre_in, n, q);
    const CnnImg im = imgs[i];
    const int iw = CIN == 16 ? im.w1 : im.w2, ow = CIN == 16 ? im.w2 : im.w4, oh = CIN == 16 ? im.h2 : im.h4;
    const int64_t ib = CIN == 16 ? im.px1 : im.px2, ob = CIN == 16 ? im.px2 : im.px4;
    const int lq = (int)(q - ib), iy = lq / iw, ix = lq - iy * iw;
    float acc = 0.f;
    if (bf(ain[q * CIN + ci]) > 0.f) {
        for (int ky = 0; ky < 3; ky++) {
            const int ty = iy + 1 - ky;
            if (ty & 1) continue;
            const int oy = ty >> 1;
            if (oy < 0 || oy >= oh) continue;
            for (int kx = 0; kx < 3; kx++) {
                const int tx = ix + 1 - kx;
                if (tx & 1) continue;
                const int ox = tx >> 1;
                if (ox < 0 || ox >= ow) continue;
                const float *gp = gout + (ob + (int64_t)oy * ow + ox) * COUT;
                const int t = ky * 3 + kx;
                for (int co = 0; co < COUT; co++) acc += gp[co] * s_w[(co * CIN + ci) * 9 + t];
            }
        }
    }
    gin[e] = acc;
}

// grad[k] = sum of the partials (fixed order); loss = sum of lz.
__global__ void cnn_reduce_kernel(const float *__restrict__ part, float *__restrict__ grad, const float *__restrict__ lz,
                                  int64_t n_lz, float *__restrict__ loss) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < CNN_NPARAM) {
        float s = 0.f;
        for (int b = 0; b < CNN_PARTS; b++) s += part[(int64_t)b * CNN_NPARAM + k];
        grad[k] = s;
    }
    if (blockIdx.x == 0 && loss) {
        __shared__ float s_l[256];
        float s = 0.f;
        for (int64_t p = threadIdx.x; p < n_lz; p += blockDim.x) s += lz[p];
        s_l[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.f;
            for (int j = 0; j < (int)blockDim.x; j++) t += s_l[j];
            loss[0] = t;
        }
    }
}

__global__ void cnn_adam_kernel(float *__restrict__ w, uint16_t *__restrict__ wb, float *__restrict__ m,
                                float *__restrict__ v, const float *__restrict__ g, int n, float lr, float b1, float b2,
                                float eps, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float wk = w[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    w[k] = wk;
    wb[k] = to_bf(wk);
}

// --------------------------------------------------------------- host side
static int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

int32_t cnn_setup(vsfe_batch *b) {
    if (b->info.n_levels < 4) return VSFE_OK;            // no level 3: the proposer is unavailable
    CnnPlan *P = new CnnPlan();
    const int n = b->n_images;
    P->n = n;
    P->h_img.resize(n);
    std::vector<int32_t> pre1(n + 1), pre2(n + 1), pre4(n + 1), pt2(n + 1), pt4(n + 1), pc(n + 1), pt1(n + 1),
        ptf(n + 1);
    int64_t s1 = 0, s2 = 0, s4 = 0, st2 = 0, st4 = 0, sc = 0, st1 = 0, stf = 0;
    for (int i = 0; i < n; i++) {
        const ImageDev &im = b->images[i];
        CnnImg &c = P->h_img[i];
        c.w0 = im.w;
        c.h0 = im.h;
        c.w3 = im.lv[3].w;
        c.h3 = im.lv[3].h;
        c.w1 = (c.w3 + 1) / 2;
        c.h1 = (c.h3 + 1) / 2;
        c.w2 = (c.w1 + 1) / 2;
        c.h2 = (c.h1 + 1) / 2;
        c.w4 = (c.w2 + 1) / 2;
        c.h4 = (c.h2 + 1) / 2;
        c.ncx0 = im.lv[0].ncx;
        c.ncy0 = im.lv[0].ncy;
        c.cell0 = im.lv[0].cell;
        c.pitch3 = im.lv[3].pitch;
        c.lvl3 = im.lv[3].offset;
        pre1[i] = (int32_t)s1;
        pre2[i] = (int32_t)s2;
        pre4[i] = (int32_t)s4;
        pt2[i] = (int32_t)st2;
        pt4[i] = (int32_t)st4;
        pc[i] = (int32_t)sc;
        pt1[i] = (int32_t)st1;
        ptf[i] = (int32_t)stf;
        c.px1 = s1;
        c.px2 = s2;
        c.px4 = s4;
        c.c0 = im.cell0_offset;
        s1 += (int64_t)c.w1 * c.h1;
        s2 += (int64_t)c.w2 * c.h2;
        s4 += (int64_t)c.w4 * c.h4;
        st2 += ((int64_t)c.w2 * c.h2 + 15) / 16;
        st4 += ((int64_t)c.w4 * c.h4 + 15) / 16;
        sc += (int64_t)c.ncx0 * c.ncy0;
        st1 += ((int64_t)c.w1 * c.h1 + 15) / 16;
        stf += (int64_t)((c.w4 + CF3W - 1) / CF3W) * ((c.h4 + CF3H - 1) / CF3H);
    }
    pre1[n] = (int32_t)s1;
    pre2[n] = (int32_t)s2;
    pre4[n] = (int32_t)s4;
    pt2[n] = (int32_t)st2;
    pt4[n] = (int32_t)st4;
    pc[n] = (int32_t)sc;
    pt1[n] = (int32_t)st1;
    ptf[n] = (int32_t)stf;
    P->px1 = s1;
    P->px2 = s2;
    P->px4 = s4;
    P->t2 = st2;
    P->t4 = st4;
    P->cells = sc;
    P->t1 = st1;
    P->tf = stf;
    for (auto *v : {&pre1, &pre2, &pre4, &pt2, &pt4, &pc, &pt1, &ptf})
        P->h_pre.insert(P->h_pre.end(), v->begin(), v->end());
    int64_t at = 0;
    P->off_wp2 = at;
    at = align256(at + 32 * 9 * 16 * 2);
    P->off_wp3 = at;
    at = align256(at + 32 * 9 * 32 * 2);
    P->off_a1 = at;
    at = align256(at + s1 * 16 * 2);
    P->off_a2 = at;
    at = align256(at + s2 * 32 * 2);
    P->off_a3 = at;
    at = align256(at + s4 * 32 * 2);
    P->off_g1 = at;
    at = align256(at + s1 * 16 * 4);
    P->off_g2 = at;
    at = align256(at + s2 * 32 * 4);
    P->off_g3 = at;
    at = align256(at + s4 * 32 * 4);
    P->off_dz = at;
    at = align256(at + s4 * 4);
    P->off_lz = at;
    at = align256(at + s4 * 4);
    P->off_part = at;
    at = align256(at + (int64_t)CNN_PARTS * CNN_NPARAM * 4);
    P->total = at;
    if (hipMalloc((void **)&P->d_img, sizeof(CnnImg) * n) != hipSuccess ||
        hipMemcpy(P->d_img, P->h_img.data(), sizeof(CnnImg) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc((void **)&P->d_pre, sizeof(int32_t) * P->h_pre.size()) != hipSuccess ||
        hipMemcpy(P->d_pre, P->h_pre.data(), sizeof(int32_t) * P->h_pre.size(), hipMemcpyHostToDevice) != hipSuccess) {
        if (P->d_img) (void)hipFree(P->d_img);
        if (P->d_pre) (void)hipFree(P->d_pre);
        delete P;
        return fail(VSFE_EHIP, "upload of the proposer tables failed");
    }
    b->cnn = P;
    b->info_cnn.workspace_bytes = P->total;
    b->info_cnn.grid_elems = s4;
    b->info_cnn.n_params = CNN_NPARAM;
    b->info_cnn.n_cells0 = sc;
    return VSFE_OK;
}

void cnn_release(vsfe_batch *b) {
    CnnPlan *P = (CnnPlan *)b->cnn;
    if (!P) return;
    if (P->d_img) (void)hipFree(P->d_img);
    if (P->d_pre) (void)hipFree(P->d_pre);
    delete P;
    b->cnn = nullptr;
}

static int32_t cnn_common(const vsfe_ctx *ctx, const vsfe_batch *b, int32_t *status, CnnPlan **P) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    *P = (CnnPlan *)b->cnn;
    if (!*P) return fail(VSFE_EINVAL, "the proposer needs at least 4 pyramid levels");
    return VSFE_OK;
}

static int32_t run_forward(const vsfe_batch *b, const CnnPlan *P, const uint8_t *pyr, const uint16_t *prm,
                           uint8_t *ws, float *z, hipStream_t st) {
    const int n = P->n;
    const int32_t *pre = P->d_pre;
    uint16_t *wp2 = (uint16_t *)(ws + P->off_wp2), *wp3 = (uint16_t *)(ws + P->off_wp3);
    uint16_t *a1 = (uint16_t *)(ws + P->off_a1), *a2 = (uint16_t *)(ws + P->off_a2), *a3 = (uint16_t *)(ws + P->off_a3);
    hipLaunchKernelGGL(cnn_pack_kernel, dim3((32 * 9 * 32 + 255) / 256), dim3(256), 0, st, prm, wp2, wp3);
    if (P->t1 > 0)
        hipLaunchKernelGGL(cnn_conv1_kernel, dim3((unsigned)((P->t1 + 3) / 4)), dim3(256), 0, st, P->d_img,
                           pre + 6 * (n + 1), n, P->t1, pyr, prm, a1);
    if (P->t2 > 0)
        hipLaunchKernelGGL((cnn_conv_mfma_kernel<16, false>), dim3((unsigned)((P->t2 + 3) / 4)), dim3(256), 0, st,
                           P->d_img, pre + 3 * (n + 1), n, P->t2, a1, a2, wp2, prm, (float *)nullptr);
    if (P->t4 > 0)
        hipLaunchKernelGGL((cnn_conv_mfma_kernel<32, true>), dim3((unsigned)((P->t4 + 3) / 4)), dim3(256), 0, st,
                           P->d_img, pre + 4 * (n + 1), n, P->t4, a2, a3, wp3, prm, z);
    (void)b;
    return check_launch("cnn forward");
}

}  // namespace vsfe

using namespace vsfe;

extern "C" {

int32_t vsfe_cnn_info_get(const vsfe_batch *b, vsfe_cnn_info *out) {
    if (!b || !out) return fail(VSFE_EINVAL, "null argument");
    if (!b->cnn) return fail(VSFE_EINVAL, "the proposer needs at least 4 pyramid levels");
    *out = b->info_cnn;
    return VSFE_OK;
}

int32_t cnn_forward(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *pyr, const uint16_t *params_bf16,
                    void *workspace, float *grid_logits, int32_t *status, void *stream) {
    CnnPlan *P = nullptr;
    int32_t rc = cnn_common(ctx, b, status, &P);
    if (rc) return rc;
    if (!pyr || !params_bf16 || !workspace || !grid_logits) return fail(VSFE_EINVAL, "null buffer");
    return run_forward(b, P, pyr, params_bf16, (uint8_t *)workspace, grid_logits, (hipStream_t)stream);
}

int32_t cnn_propose(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *pyr, const uint16_t *params_bf16,
                    float thresh, void *workspace, float *grid_logits, float *cell_logits, uint8_t *cell_mask,
                    int32_t *status, void *stream) {
    CnnPlan *P = nullptr;
    int32_t rc = cnn_common(ctx, b, status, &P);
    if (rc) return rc;
    if (!pyr || !params_bf16 || !workspace || !grid_logits || !cell_mask) return fail(VSFE_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    uint8_t *ws = (uint8_t *)workspace;
    uint16_t *wp2 = (uint16_t *)(ws + P->off_wp2), *wp3 = (uint16_t *)(ws + P->off_wp3);
    hipLaunchKernelGGL(cnn_pack_kernel, dim3((32 * 9 * 32 + 255) / 256), dim3(256), 0, st, params_bf16, wp2, wp3);
    if (P->tf > 0)
        hipLaunchKernelGGL(cnn_fused_fwd_kernel, dim3((unsigned)P->tf), dim3(256), 0, st, P->d_img,
                           P->d_pre + 7 * (P->n + 1), P->n, pyr, params_bf16, wp2, wp3, grid_logits);
    rc = check_launch("cnn_propose (forward)");
    if (rc) return rc;
    if (P->cells > 0)
        hipLaunchKernelGGL(cnn_cells_kernel, dim3((unsigned)((P->cells + 255) / 256)), dim3(256), 0, st, P->d_img,
                           P->d_pre + 5 * (P->n + 1), P->n, P->cells, grid_logits, thresh, cell_logits, cell_mask,
                           ctx->scale_q16[3]);
    return check_launch("cnn_propose");
}

int32_t cnn_backward(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *pyr, const uint16_t *params_bf16,
                     void *workspace, const float *grid_logits, const float *grid_targets, float pos_weight,
                     float *grad, float *loss, int32_t *status, void *stream) {
    CnnPlan *P = nullptr;
    int32_t rc = cnn_common(ctx, b, status, &P);
    if (rc) return rc;
    if (!pyr || !params_bf16 || !workspace || !grid_logits || !grid_targets || !grad)
        return fail(VSFE_EINVAL, "null buffer");
    if (!(pos_weight > 0.f)) return fail(VSFE_EINVAL, "pos_weight must be positive");
    hipStream_t st = (hipStream_t)stream;
    uint8_t *ws = (uint8_t *)workspace;
    const int n = P->n;
    const int32_t *pre = P->d_pre;
    uint16_t *a1 = (uint16_t *)(ws + P->off_a1), *a2 = (uint16_t *)(ws + P->off_a2), *a3 = (uint16_t *)(ws + P->off_a3);
    float *g1 = (float *)(ws + P->off_g1), *g2 = (float *)(ws + P->off_g2), *g3 = (float *)(ws + P->off_g3);
    float *dz = (float *)(ws + P->off_dz), *lz = (float *)(ws + P->off_lz), *part = (float *)(ws + P->off_part);
    if (P->px4 <= 0) return fail(VSFE_EINVAL, "empty proposer grid");
    hipLaunchKernelGGL(cnn_head_bwd_kernel, dim3((unsigned)((P->px4 + 255) / 256)), dim3(256), 0, st, P->px4,
                       grid_logits, grid_targets, pos_weight, params_bf16, a3, dz, lz, g3);
    hipLaunchKernelGGL(cnn_head_wgrad_kernel, dim3(CNN_PARTS), dim3(256), 0, st, P->px4, dz, a3, part);
    hipLaunchKernelGGL((cnn_wgrad_kernel<32, 32, false>), dim3(CNN_PARTS, 4), dim3(256), 0, st, P->d_img,
                       pre + 2 * (n + 1), n, P->px4, g3, a2, pyr, part, P_W3, P_B3);
    hipLaunchKernelGGL((cnn_dgrad_kernel<32, 32>), dim3((unsigned)((P->px2 * 32 + 255) / 256)), dim3(256), 0, st,
                       P->d_img, pre + 1 * (n + 1), n, P->px2, g3, a2, params_bf16, P_W3, g2);
    hipLaunchKernelGGL((cnn_wgrad_kernel<16, 32, false>), dim3(CNN_PARTS, 2), dim3(256), 0, st, P->d_img,
                       pre + 1 * (n + 1), n, P->px2, g2, a1, pyr, part, P_W2, P_B2);
    hipLaunchKernelGGL((cnn_dgrad_kernel<16, 32>), dim3((unsigned)((P->px1 * 16 + 255) / 256)), dim3(256), 0, st,
                       P->d_img, pre, n, P->px1, g2, a1, params_bf16, P_W2, g1);
    hipLaunchKernelGGL((cnn_wgrad_kernel<1, 16, true>), dim3(CNN_PARTS), dim3(256), 0, st, P->d_img, pre, n, P->px1,
                       g1, a1, pyr, part, P_W1, P_B1);
    hipLaunchKernelGGL(cnn_reduce_kernel, dim3((CNN_NPARAM + 255) / 256), dim3(256), 0, st, part, grad, lz, P->px4,
                       loss);
    return check_launch("cnn_backward");
}

int32_t cnn_adam_step(float *params, uint16_t *params_bf16, float *m, float *v, const float *grad, int32_t n,
                      float lr, float beta1, float beta2, float eps, int32_t step, void *stream) {
    if (!params || !params_bf16 || !m || !v || !grad) return fail(VSFE_EINVAL, "null buffer");
    if (n < 1 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f))
        return fail(VSFE_EINVAL, "bad optimizer arguments");
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(cnn_adam_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, params_bf16,
                       m, v, grad, n, lr, beta1, beta2, eps, c1, c2);
    return check_launch("cnn_adam_step");
}

}  // extern "C"
