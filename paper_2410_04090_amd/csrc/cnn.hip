// Learned cell proposer: a small CNN on pyramid level 3 that predicts which
// native-scale cells will hold final keypoints, so the exact detector runs
// only there (the gating itself is in fast_br_detect).
//
// Network (one logit per stride-8 position of level 3):
//   x = (I_3 - 128) / 128 -> conv3x3 s2 (1 -> 16) -> ReLU -> conv3x3 s2
//   (16 -> 32) -> ReLU -> conv3x3 s2 (32 -> 32) -> ReLU -> conv1x1 (32 -> 1).
// Padding 1, ceil(in / 2) outputs per axis.  Parameters are one flat
// vector, OIHW weights followed by biases per layer; the kernels read its
// bfloat16 copy, so the network evaluated is the bfloat16-valued one.
//
// Precision.  The input (I - 128) / 128 and the weights are exact in both
// half formats.  Every product runs on the matrix cores with float32
// accumulation; what differs is how an activation enters the next layer:
//  * inference (cnn_propose) stores it as float16 (11 significant bits):
//    the logits of the packaged trained networks stay within 5e-3 of a
//    float64 forward (a single bfloat16 would give up to 0.03);
//  * training (cnn_forward, before cnn_backward) keeps float32 activations
//    and feeds each convolution a bfloat16 value and remainder pair (hi +
//    lo, about 16 significant bits) in separate accumulator chains, so the
//    gradients see logits within about 1e-4 of float32.
// The 1x1 head reads conv3's float32 output directly in both.
//
//  * conv1 (K = 9 taps) runs on the 16x16x16 matrix instruction: lane
//    group g takes tap row g as the K slots (input columns 2x - 2 .. 2x + 1,
//    the first with a zero weight);
//  * conv2 (K = 144) and conv3 (K = 288) are implicit GEMMs on the
//    16x16x32 instruction (conv2's ninth tap on 16x16x16): weights are the
//    A operand (row = output channel), activations the B operand (column =
//    output pixel, 8 channels of one tap per lane);
//  * inference runs the three layers and the head fused in one persistent
//    kernel over 6 x 7 tiles of grid positions (activations in LDS, conv1
//    and conv2 in even / odd column planes so that the stride-2 reads of
//    the next layer take consecutive entries).  Two phases per tile: conv1
//    of tile k beside conv3 + head of tile k - 1, then conv2 of tile k
//    beside the staging of tile k + 1, whose input was fetched a phase
//    earlier, and the fetch of tile k + 2;
//  * cell logits: per native-scale cell, the maximum over the grid
//    positions whose projected centre ((8 j + 4) S_3 + 2^15) >> 16 falls in
//    it (a cell with none is always kept);
//  * training: mean binary cross-entropy with a positive-class weight,
//    backward in float32 on the VALU, weight gradients as per-block partial
//    sums reduced in a fixed order (deterministic), then Adam.
#include <string.h>

#include <algorithm>
#include <type_traits>

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
    int64_t off_wp2 = 0, off_wp3 = 0, off_hp1 = 0, off_hp2 = 0, off_hp3 = 0, off_a1 = 0, off_a2 = 0, off_a3 = 0, off_g1 = 0, off_g2 = 0, off_g3 = 0,
            off_dz = 0, off_lz = 0, off_part = 0, total = 0;
};


typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf(uint16_t v) { return __builtin_bit_cast(float, (uint32_t)v << 16); }
__device__ __forceinline__ uint16_t to_bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ f32x4 relu4(f32x4 v) {
    f32x4 r;
#pragma unroll
    for (int i = 0; i < 4; i++) r[i] = fmaxf(v[i], 0.0f);
    return r;
}

// the input (I - 128) / 128 of byte b of v: exact in float32, bfloat16 and float16
__device__ __forceinline__ float x_byte(uint32_t v, int b) {
    return fmaf((float)((v >> (8 * b)) & 255u), 1.0f / 128.0f, -1.0f);
}

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

__device__ __forceinline__ f32x4 splat4(float v) {
    const f32x4 r = {v, v, v, v};
    return r;
}

// per-lane biases (the accumulator's start): channels at + 4 g .. + 3
__device__ __forceinline__ f32x4 conv_bias(const uint16_t *prm, int at, int lane) {
    const int g = lane >> 4;
    f32x4 b;
#pragma unroll
    for (int r = 0; r < 4; r++) b[r] = bf(prm[at + 4 * g + r]);
    return b;
}

// MFMA lane layout (16 x 16 output tiles): lane l works on output pixel
// l % 16 and K slice g = l / 16; its accumulator holds output channels
// 4 g .. 4 g + 3 of its 16-channel block.

// Repack the weights: bfloat16 conv2 / conv3 as [co][tap][ci] for the
// training forward, and float16 copies for inference (saturated to the
// largest finite float16): conv1 [g][c][4] (lane c + 16 g: tap row g of
// channel c as K slots (0, w[g][0], w[g][1], w[g][2]), group 3 zero), conv2
// and conv3 [co][tap][ci].
__global__ void cnn_pack_kernel(const uint16_t *__restrict__ prm, uint16_t *__restrict__ wp2, uint16_t *__restrict__ wp3,
                                uint16_t *__restrict__ hp1, uint16_t *__restrict__ hp2, uint16_t *__restrict__ hp3) {
    auto to_h = [](float f) { return __builtin_bit_cast(uint16_t, (_Float16)fminf(fmaxf(f, -65504.f), 65504.f)); };
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 16 * 4 * 4) {
        const int g = i / 64, c = (i / 4) % 16, s = i % 4;
        hp1[i] = (g < 3 && s > 0) ? to_h(bf(prm[P_W1 + c * 9 + g * 3 + s - 1])) : (uint16_t)0;
    }
    if (i < 32 * 9 * 16) {
        const int co = i / (9 * 16), t = (i / 16) % 9, ci = i % 16;
        const uint16_t w = prm[P_W2 + (co * 16 + ci) * 9 + t];
        wp2[i] = w;
        hp2[i] = to_h(bf(w));
    }
    if (i < 32 * 9 * 32) {
        const int co = i / (9 * 32), t = (i / 32) % 9, ci = i % 32;
        const uint16_t w = prm[P_W3 + (co * 32 + ci) * 9 + t];
        wp3[i] = w;
        hp3[i] = to_h(bf(w));
    }
}

// ---- training forward (cnn_forward): layer by layer through HBM with
// float32 activations, each convolution input carried as a bfloat16 value
// + remainder pair (hi + lo, about 16 significant bits) on the bfloat16
// matrix cores, so that the gradients of the training loop see logits
// within about 1e-4 of a float32 forward
namespace tr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf_lo(uint32_t v) { return __builtin_bit_cast(float, v << 16); }
__device__ __forceinline__ float bf_hi(uint32_t v) { return __builtin_bit_cast(float, v & 0xFFFF0000u); }

// two floats as packed bfloat16 (round to nearest even): v_cvt_pk_bf16_f32
__device__ __forceinline__ uint32_t pk_bf(float a, float b) {
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// value / remainder pair of two activations: hi = bf16(v), lo = bf16(v - hi)
__device__ __forceinline__ void split2(float a, float b, uint32_t *hi, uint32_t *lo) {
    const uint32_t h = pk_bf(a, b);
    *hi = h;
    *lo = pk_bf(a - bf_lo(h), b - bf_hi(h));
}

// 4 activations (one lane's accumulator after bias and ReLU) as hi / lo pairs
__device__ __forceinline__ void split4(f32x4 v, uint2 *hi, uint2 *lo) {
    split2(v[0], v[1], &hi->x, &lo->x);
    split2(v[2], v[3], &hi->y, &lo->y);
}

// 8 float32 activations as hi / lo bfloat16x8 operands
__device__ __forceinline__ void split8(float4 a, float4 b, uint4 *hi, uint4 *lo) {
    split2(a.x, a.y, &hi->x, &lo->x);
    split2(a.z, a.w, &hi->y, &lo->y);
    split2(b.x, b.y, &hi->z, &lo->z);
    split2(b.z, b.w, &hi->w, &lo->w);
}

__device__ __forceinline__ f32x4 mfma16(i16x4 a, i16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(uint4 a, uint4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                  0);
}
__device__ __forceinline__ i16x4 as_i16x4(uint2 v) { return __builtin_bit_cast(i16x4, v); }

// conv1 A operand: lane (channel c = l % 16, group g = l / 16).  Group g < 3
// holds tap row g as K slots (0, w[g][0], w[g][1], w[g][2]); group 3 is zero.
__device__ __forceinline__ i16x4 conv1_a(const uint16_t *prm, int lane) {
    const int c = lane & 15, g = lane >> 4;
    i16x4 w = {0, 0, 0, 0};
    if (g < 3) {
#pragma unroll
        for (int kx = 0; kx < 3; kx++) w[kx + 1] = (short)prm[P_W1 + c * 9 + g * 3 + kx];
    }
    return w;
}

// Weights of one 16-channel block (rows co0 .. co0 + 15) of conv2: four
// 32-wide K chunks (taps 2c and 2c + 1, 16 channels each; lane group g takes
// tap 2c + g / 2, channels 8 (g & 1) .. + 7) and tap 8 on 16 K (channels
// 4 g .. 4 g + 3).
struct W2 {
    uint4 c[4];
    uint2 t8;
};
__device__ __forceinline__ W2 conv2_a(const uint16_t *wp2, int lane, int co0) {
    const int m = lane & 15, g = lane >> 4;
    W2 w;
#pragma unroll
    for (int c = 0; c < 4; c++) w.c[c] = *(const uint4 *)(wp2 + ((co0 + m) * 9 + 2 * c + (g >> 1)) * 16 + 8 * (g & 1));
    w.t8 = *(const uint2 *)(wp2 + ((co0 + m) * 9 + 8) * 16 + 4 * g);
    return w;
}

// conv3 weights of one 16-channel block: tap t, lane group g -> channels 8 g .. 8 g + 7
struct W3 {
    uint4 t[9];
};
__device__ __forceinline__ W3 conv3_a(const uint16_t *wp3, int lane, int co0) {
    const int m = lane & 15, g = lane >> 4;
    W3 w;
#pragma unroll
    for (int t = 0; t < 9; t++) w.t[t] = *(const uint4 *)(wp3 + ((co0 + m) * 9 + t) * 32 + 8 * g);
    return w;
}

// B operands of one conv2 output pixel (per lane: its K slice), value and
// remainder parts
struct B2 {
    uint4 h[4], l[4];
    uint2 h8, l8;
};
struct B3 {
    uint4 h[9], l[9];
};

// conv2 on the pair chains of both 16-channel blocks (hi chain from the
// bias, lo chain from zero, tap by tap, then hi + lo)
__device__ __forceinline__ void conv2_mfma(const W2 &wa, const W2 &wb, const B2 &b, f32x4 bias_a, f32x4 bias_b,
                                           f32x4 *va, f32x4 *vb) {
    f32x4 ah = bias_a, bh = bias_b, al = splat4(0.f), bl = splat4(0.f);
#pragma unroll
    for (int c = 0; c < 4; c++) {
        ah = mfma32(wa.c[c], b.h[c], ah);
        bh = mfma32(wb.c[c], b.h[c], bh);
        al = mfma32(wa.c[c], b.l[c], al);
        bl = mfma32(wb.c[c], b.l[c], bl);
    }
    ah = mfma16(as_i16x4(wa.t8), as_i16x4(b.h8), ah);
    bh = mfma16(as_i16x4(wb.t8), as_i16x4(b.h8), bh);
    al = mfma16(as_i16x4(wa.t8), as_i16x4(b.l8), al);
    bl = mfma16(as_i16x4(wb.t8), as_i16x4(b.l8), bl);
    *va = mfma_settle(ah) + mfma_settle(al);
    *vb = mfma_settle(bh) + mfma_settle(bl);
}

// conv3 of one 16-channel block
__device__ __forceinline__ f32x4 conv3_mfma(const W3 &w, const B3 &b, f32x4 bias) {
    f32x4 h = bias, l = splat4(0.f);
#pragma unroll
    for (int t = 0; t < 9; t++) {
        h = mfma32(w.t[t], b.h[t], h);
        l = mfma32(w.t[t], b.l[t], l);
    }
    return mfma_settle(h) + mfma_settle(l);
}

// 1x1 head partial of one 16-channel block (after ReLU): sum over the
// lane's 4 channels, then over the 4 lane groups (fixed order); every lane
// of column m ends with the block's sum for pixel m
__device__ __forceinline__ float head16(f32x4 a, const uint16_t *prm, int co0, int lane) {
    const int g = lane >> 4;
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < 4; r++) s = fmaf(bf(prm[P_W4 + co0 + 4 * g + r]), a[r], s);
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s;
}

// ---- layer-by-layer kernels (training): one wave = 16 consecutive output
// pixels of one image (row-major), float32 NHWC activations

__global__ __launch_bounds__(256) void cnn_conv1_kernel(const CnnImg *__restrict__ imgs,
                                                        const int32_t *__restrict__ pre_tiles, int n,
                                                        int64_t total_tiles, const uint8_t *__restrict__ pyr,
                                                        const uint16_t *__restrict__ prm, float *__restrict__ a1) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile >= total_tiles) return;
    const int i = find_image(pre_tiles, n, tile);
    const CnnImg im = imgs[i];
    const int npx = im.w1 * im.h1;
    const int m = lane & 15, g = lane >> 4;
    const int pm = (int)(tile - pre_tiles[i]) * 16 + m;
    const int oy = pm / im.w1, ox = pm - oy * im.w1;
    // K slots of group g: tap row g, input columns 2 ox - 2 .. 2 ox + 1
    float x[4] = {0.f, 0.f, 0.f, 0.f};
    const int iy = 2 * oy + (g < 3 ? g : 2) - 1;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int ix = 2 * ox - 2 + j;
        if (pm < npx && g < 3 && iy >= 0 && iy < im.h3 && ix >= 0 && ix < im.w3) {
            const uint32_t v = pyr[im.lvl3 + (int64_t)iy * im.pitch3 + ix];
            x[j] = x_byte(v, 0);
        }
    }
    const uint2 xb = make_uint2(pk_bf(x[0], x[1]), pk_bf(x[2], x[3]));
    const f32x4 acc = relu4(mfma_settle(mfma16(conv1_a(prm, lane), as_i16x4(xb), conv_bias(prm, P_B1, lane))));
    if (pm < npx) *(f32x4 *)(a1 + (im.px1 + pm) * 16 + 4 * g) = acc;
}

// 8 float32 channels at (y, x) of an NHWC map, zero outside
__device__ __forceinline__ void load8(const float *a, int C, int64_t base, int w, int h, int y, int x, int ci0,
                                      bool ok, float4 *p, float4 *q) {
    *p = make_float4(0.f, 0.f, 0.f, 0.f);
    *q = *p;
    if (ok && y >= 0 && y < h && x >= 0 && x < w) {
        const float *s = a + (base + (int64_t)y * w + x) * C + ci0;
        *p = *(const float4 *)s;
        *q = *(const float4 *)(s + 4);
    }
}

__global__ __launch_bounds__(256) void cnn_conv2_kernel(const CnnImg *__restrict__ imgs,
                                                        const int32_t *__restrict__ pre_tiles, int n,
                                                        int64_t total_tiles, const float *__restrict__ a1,
                                                        float *__restrict__ a2, const uint16_t *__restrict__ wp2,
                                                        const uint16_t *__restrict__ prm) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile >= total_tiles) return;
    const int i = find_image(pre_tiles, n, tile);
    const CnnImg im = imgs[i];
    const int npx = im.w2 * im.h2;
    const int m = lane & 15, g = lane >> 4;
    const int pm = (int)(tile - pre_tiles[i]) * 16 + m;
    const bool valid = pm < npx;
    const int oy = valid ? pm / im.w2 : 0, ox = valid ? pm - oy * im.w2 : 0;
    B2 b;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const int t = 2 * c + (g >> 1);
        float4 p, q;
        load8(a1, 16, im.px1, im.w1, im.h1, 2 * oy + t / 3 - 1, 2 * ox + t % 3 - 1, 8 * (g & 1), valid, &p, &q);
        split8(p, q, &b.h[c], &b.l[c]);
    }
    {
        float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
        const int y = 2 * oy + 1, x = 2 * ox + 1;
        if (valid && y < im.h1 && x < im.w1) p = *(const float4 *)(a1 + (im.px1 + (int64_t)y * im.w1 + x) * 16 + 4 * g);
        split2(p.x, p.y, &b.h8.x, &b.l8.x);
        split2(p.z, p.w, &b.h8.y, &b.l8.y);
    }
    const W2 wa = conv2_a(wp2, lane, 0), wb = conv2_a(wp2, lane, 16);
    f32x4 va, vb;
    conv2_mfma(wa, wb, b, conv_bias(prm, P_B2, lane), conv_bias(prm, P_B2 + 16, lane), &va, &vb);
    if (valid) {
        float *o = a2 + (im.px2 + pm) * 32 + 4 * g;
        *(f32x4 *)o = relu4(va);
        *(f32x4 *)(o + 16) = relu4(vb);
    }
}

__global__ __launch_bounds__(256) void cnn_conv3_kernel(const CnnImg *__restrict__ imgs,
                                                        const int32_t *__restrict__ pre_tiles, int n,
                                                        int64_t total_tiles, const float *__restrict__ a2,
                                                        float *__restrict__ a3, const uint16_t *__restrict__ wp3,
                                                        const uint16_t *__restrict__ prm, float *__restrict__ z) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + wave;
    if (tile >= total_tiles) return;
    const int i = find_image(pre_tiles, n, tile);
    const CnnImg im = imgs[i];
    const int npx = im.w4 * im.h4;
    const int m = lane & 15, g = lane >> 4;
    const int pm = (int)(tile - pre_tiles[i]) * 16 + m;
    const bool valid = pm < npx;
    const int oy = valid ? pm / im.w4 : 0, ox = valid ? pm - oy * im.w4 : 0;
    B3 b;
#pragma unroll
    for (int t = 0; t < 9; t++) {
        float4 p, q;
        load8(a2, 32, im.px2, im.w2, im.h2, 2 * oy + t / 3 - 1, 2 * ox + t % 3 - 1, 8 * g, valid, &p, &q);
        split8(p, q, &b.h[t], &b.l[t]);
    }
    f32x4 v0, v1;
    {
        const W3 w = conv3_a(wp3, lane, 0);
        v0 = relu4(conv3_mfma(w, b, conv_bias(prm, P_B3, lane)));
    }
    {
        const W3 w = conv3_a(wp3, lane, 16);
        v1 = relu4(conv3_mfma(w, b, conv_bias(prm, P_B3 + 16, lane)));
    }
    // head: block 0's sum plus block 1's, then the bias (fixed order)
    const float part = head16(v0, prm, 0, lane) + head16(v1, prm, 16, lane);
    if (valid) {
        float *o = a3 + (im.px4 + pm) * 32 + 4 * g;
        *(f32x4 *)o = v0;
        *(f32x4 *)(o + 16) = v1;
        if (g == 0) z[im.px4 + pm] = part + bf(prm[P_B4]);
    }
}

}  // namespace tr

// ---- inference (cnn_propose): activations stored as float16 (11
// significant bits) on the float16 matrix cores, float32 sums
namespace inf {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));


// two floats as packed float16, round to nearest even (v_cvt_pk_f16_f32)
__device__ __forceinline__ uint32_t pk_h(float a, float b) {
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
}

// ReLU of a packed float16 pair (after rounding: max(round(x), 0) equals
// round(max(x, 0)) up to the sign of zero)
__device__ __forceinline__ uint32_t relu_h2(uint32_t v) {
    const f16x2 z = {(_Float16)0.f, (_Float16)0.f};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(f16x2, v), z));
}

// 4 accumulator values after ReLU as float16
__device__ __forceinline__ uint2 relu_h4(f32x4 v) {
    return make_uint2(relu_h2(pk_h(v[0], v[1])), relu_h2(pk_h(v[2], v[3])));
}

// 8 float32 activations (already >= 0) as float16
__device__ __forceinline__ uint4 h8(float4 a, float4 b) {
    return make_uint4(pk_h(a.x, a.y), pk_h(a.z, a.w), pk_h(b.x, b.y), pk_h(b.z, b.w));
}

// (I - 128) / 128 of the four bytes of v as two float16 pairs: the half
// with bits 0x6400 | I is 1024 + I, and (1024 + I) / 128 - 9 is exact
__device__ __forceinline__ uint2 x_h4(uint32_t v) {
    const f16x2 s = {(_Float16)0.0078125f, (_Float16)0.0078125f}, o = {(_Float16)-9.f, (_Float16)-9.f};
    const f16x2 a = __builtin_bit_cast(f16x2, __builtin_amdgcn_perm(v, 0x64646464u, 0x00050004u));
    const f16x2 b = __builtin_bit_cast(f16x2, __builtin_amdgcn_perm(v, 0x64646464u, 0x00070006u));
    return make_uint2(__builtin_bit_cast(uint32_t, __builtin_elementwise_fma(a, s, o)),
                      __builtin_bit_cast(uint32_t, __builtin_elementwise_fma(b, s, o)));
}

__device__ __forceinline__ f32x4 mfma16(uint2 a, uint2 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(f16x4, a), __builtin_bit_cast(f16x4, b), c, 0, 0,
                                                 0);
}
__device__ __forceinline__ f32x4 mfma32(uint4 a, uint4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0,
                                                 0);
}

// conv1 A operand of a lane (channel l % 16, tap row l / 16)
__device__ __forceinline__ uint2 conv1_a(const uint16_t *wp1, int lane) {
    return *(const uint2 *)(wp1 + 4 * lane);
}

// Weights of one 16-channel block (rows co0 .. co0 + 15) of conv2: four
// 32-wide K chunks (taps 2c and 2c + 1, 16 channels each; lane group g takes
// tap 2c + g / 2, channels 8 (g & 1) .. + 7) and tap 8 on 16 K (channels
// 4 g .. 4 g + 3).
struct W2 {
    uint4 c[4];
    uint2 t8;
};
__device__ __forceinline__ W2 conv2_a(const uint16_t *wp2, int lane, int co0) {
    const int m = lane & 15, g = lane >> 4;
    W2 w;
#pragma unroll
    for (int c = 0; c < 4; c++) w.c[c] = *(const uint4 *)(wp2 + ((co0 + m) * 9 + 2 * c + (g >> 1)) * 16 + 8 * (g & 1));
    w.t8 = *(const uint2 *)(wp2 + ((co0 + m) * 9 + 8) * 16 + 4 * g);
    return w;
}

// conv3 weights of one 16-channel block: tap t, lane group g -> channels 8 g .. 8 g + 7
struct W3 {
    uint4 t[9];
};
__device__ __forceinline__ W3 conv3_a(const uint16_t *wp3, int lane, int co0) {
    const int m = lane & 15, g = lane >> 4;
    W3 w;
#pragma unroll
    for (int t = 0; t < 9; t++) w.t[t] = *(const uint4 *)(wp3 + ((co0 + m) * 9 + t) * 32 + 8 * g);
    return w;
}

// B operands of one conv2 output pixel (per lane: its K slice)
struct B2 {
    uint4 c[4];
    uint2 t8;
};

// one 16-channel block of conv2 / conv3: the bias starts the chain, then
// the K chunks in tap order (the same order in the fused and the
// layer-by-layer kernels)
__device__ __forceinline__ f32x4 conv2_mfma(const W2 &w, const B2 &b, f32x4 bias) {
    f32x4 acc = bias;
#pragma unroll
    for (int c = 0; c < 4; c++) acc = mfma32(w.c[c], b.c[c], acc);
    return mfma16(w.t8, b.t8, acc);
}

// 1x1 head weights of a lane's 4 channels in block co0
__device__ __forceinline__ f32x4 head_w(const uint16_t *prm, int co0, int lane) {
    return conv_bias(prm, P_W4 + co0, lane);
}

// 1x1 head partial of one 16-channel block (after ReLU): sum over the
// lane's 4 channels, then over the 4 lane groups (fixed order); every lane
// of column m ends with the block's sum for pixel m
__device__ __forceinline__ float head16(f32x4 a, f32x4 w) {
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < 4; r++) s = fmaf(w[r], a[r], s);
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s;
}

// ---- fused inference forward: a persistent 256-thread block walks 6 x 7
// tiles of grid positions with every activation in LDS (float16).  Windows
// (rows x columns) of a tile at grid (Y3, X3): conv2 13 x 15 from
// (2 Y3 - 1, 2 X3 - 1), conv1 27 x 31, input 55 x 68 from (8 Y3 - 7,
// 8 X3 - 8); positions outside an activation map are its zero padding.
// conv1 and conv2 are stored in even / odd column planes (entry = (parity,
// row, column pair)) so that the stride-2 reads of the next layer take 16
// consecutive entries; each plane has one pad column, never read.
//
// Work per tile (4 waves):
//  * conv1: unit = (row, parity), 16 pixels x 16 channels; wave w has
//    parity w & 1 and rows 0..11 (w < 2) or 12..26 (w >= 2);
//  * conv2: unit = one row (15 pixels) x both 16-channel blocks, so every
//    operand read from LDS feeds two products; wave w has rows w + 4 i;
//  * conv3 + head: unit = (16 positions, one 16-channel block); wave w has
//    block w & 1 and position groups (w >> 1) + 2 i (two for waves 0 and 1,
//    one for waves 2 and 3, which take three more conv1 units instead).
constexpr int F3H = 6, F3W = 7;
constexpr int F2H = 2 * F3H + 1, F2W = 2 * F3W + 1;      // 13 x 15
constexpr int F1H = 2 * F2H + 1, F1W = 2 * F2W + 1;      // 27 x 31
constexpr int F0H = 2 * F1H + 1;                         // 55 input rows
constexpr int F1J = 16, F2J = 8;                         // column pairs per plane
static_assert(2 * F1J == F1W + 1 && 2 * F2J == F2W + 1, "one pad column per plane");
constexpr int F0D = 17;                                  // input dwords per row (68 columns)
constexpr int F0S = 8 * F0D;                             // staged row stride (bytes, float16)
// conv1 planes: row = 2 halves (8 channels) x 16 pairs of 16 bytes, so the
// 16 lanes of a K slice read 16 consecutive chunks; conv2 planes: row = 4
// quarters x 8 pairs of 16 bytes plus 64 bytes of padding, so that the two
// grid rows one conv3 tile reads (conv2 rows 2 apart) fall on disjoint banks
constexpr int RS1 = 2 * F1J * 16, RS2 = 4 * F2J * 16 + 64;     // row strides (bytes)
// conv2's odd-column plane starts 128 bytes off the even one's banks, so the
// even and odd output columns a conv2 unit writes do not share banks
constexpr int P2 = F2H * RS2 + 64;                       // conv2 plane stride (bytes)
static_assert(P2 % 256 == 128, "conv2 planes half a bank period apart");
constexpr int A1B = 2 * F1H * RS1, A2B = 2 * P2;         // plane pairs (bytes)
constexpr int F_WAVES = 4, F_THREADS = 64 * F_WAVES;
constexpr int F_LD = (F0H * F0D + F_THREADS - 1) / F_THREADS;   // input dwords per thread (4)
constexpr int F_NPOS = F3H * F3W;                        // 42 grid positions
constexpr int F_R1A = 12, F_R1B = F1H - F_R1A;           // conv1 rows of waves 0, 1 / 2, 3
constexpr int F_NT = (F_NPOS + 15) / 16;                 // conv3 position groups (3)
constexpr int F_BLOCKS_PER_CU = 3;
static_assert(F_R1B - F_R1A == 3 && F_NT == 3, "the conv1 / conv3 balance below assumes these counts");

// geometry of one tile: its image and grid origin (uniform)
struct FTile {
    int img, Y3, X3;
};

__device__ __forceinline__ FTile fused_tile(const CnnImg *imgs, const int32_t *pre, int n, int t, int &cursor) {
    while (cursor + 1 < n && pre[cursor + 1] <= t) cursor++;
    const CnnImg &im = imgs[cursor];
    const int ntx = (im.w4 + F3W - 1) / F3W;
    const int lt = t - pre[cursor], ty = lt / ntx;
    return FTile{cursor, ty * F3H, (lt - ty * ntx) * F3W};
}

// the input dwords of a tile this thread stages (zero outside the level)
__device__ __forceinline__ void fused_fetch(const uint8_t *pyr, const CnnImg &im, const FTile &f, const int *rr,
                                            const int *jj, uint32_t *v) {
    const int Y0 = 8 * f.Y3 - 7, XS = 8 * f.X3 - 8;
    const uint8_t *base = pyr + im.lvl3;
    const bool interior = Y0 >= 0 && Y0 + F0H <= im.h3 && XS >= 0 && XS + 4 * F0D <= im.w3;
    if (interior) {
#pragma unroll
        for (int k = 0; k < F_LD; k++)
            v[k] = rr[k] < F0H ? *(const uint32_t *)(base + (uint32_t)((Y0 + rr[k]) * im.pitch3 + XS + 4 * jj[k])) : 0u;
    } else {
#pragma unroll
        for (int k = 0; k < F_LD; k++) {
            const int gy = Y0 + rr[k], gx = XS + 4 * jj[k];
            const bool ok = rr[k] < F0H && gy >= 0 && gy < im.h3 && gx >= 0 && gx < im.w3;
            v[k] = ok ? *(const uint32_t *)(base + (uint32_t)(gy * im.pitch3 + gx)) : 0u;
        }
    }
}

// stage fetched dwords as float16 (I - 128) / 128, zero outside the level
__device__ __forceinline__ void fused_stage(uint8_t *s_in, const CnnImg &im, const FTile &f, const int *rr,
                                            const int *jj, const uint32_t *v) {
    const int Y0 = 8 * f.Y3 - 7, XS = 8 * f.X3 - 8;
    const bool interior = Y0 >= 0 && Y0 + F0H <= im.h3 && XS >= 0 && XS + 4 * F0D <= im.w3;
#pragma unroll
    for (int k = 0; k < F_LD; k++) {
        if (rr[k] >= F0H) continue;
        uint2 x = x_h4(v[k]);
        if (!interior) {
            const int gy = Y0 + rr[k], gx = XS + 4 * jj[k];
            const bool row = gy >= 0 && gy < im.h3 && gx >= 0;
            const int nv = row ? min(max(im.w3 - gx, 0), 4) : 0;       // valid columns of the dword
            x.x &= nv >= 2 ? 0xFFFFFFFFu : (nv == 1 ? 0xFFFFu : 0u);
            x.y &= nv >= 4 ? 0xFFFFFFFFu : (nv == 3 ? 0xFFFFu : 0u);
        }
        *(uint2 *)(s_in + rr[k] * F0S + 8 * jj[k]) = x;
    }
}

// bit r set for the window rows r in [lo, hi)
__device__ __forceinline__ uint32_t row_bits(int lo, int hi) {
    lo = max(lo, 0);
    return hi > lo ? (hi >= 32 ? 0xFFFFFFFFu : (1u << hi) - 1u) & ~((1u << lo) - 1u) : 0u;
}

__global__ __launch_bounds__(F_THREADS, F_BLOCKS_PER_CU) void cnn_fused_fwd_kernel(
    const CnnImg *__restrict__ imgs, const int32_t *__restrict__ pre_tiles, int n, int n_tiles,
    const uint8_t *__restrict__ pyr, const uint16_t *__restrict__ prm, const uint16_t *__restrict__ wp1,
    const uint16_t *__restrict__ wp2, const uint16_t *__restrict__ wp3, float *__restrict__ z) {
    __shared__ __attribute__((aligned(16))) uint8_t s_in[F0H * F0S];
    __shared__ uint4 s_a1[A1B / 16];
    __shared__ uint4 s_a2[A2B / 16];
    __shared__ float s_head[2][16 * F_NT];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int m = lane & 15, g = lane >> 4;

    // this block's tiles: XCD x = block % 8 owns a contiguous eighth of the
    // tiles, which its blocks take in turn (neighbouring tiles share halo
    // rows in that XCD's L2)
    const int x = blockIdx.x % N_XCD, nbx = ((int)gridDim.x - x + N_XCD - 1) / N_XCD, lb = blockIdx.x / N_XCD;
    const int t_lo = (int)((int64_t)n_tiles * x / N_XCD), t_hi = (int)((int64_t)n_tiles * (x + 1) / N_XCD);
    const int first = t_lo + lb;
    const int K = first < t_hi ? (t_hi - first + nbx - 1) / nbx : 0;
    if (K == 0) return;
    auto tile_at = [&](int k) { return first + k * nbx; };

    // staging slots of this thread (tile independent)
    int rr[F_LD], jj[F_LD];
#pragma unroll
    for (int k = 0; k < F_LD; k++) {
        const int d = tid + F_THREADS * k;
        rr[k] = d / F0D;                                  // >= F0H: no slot
        jj[k] = d - rr[k] * F0D;
    }

    // weights held for the whole walk
    const uint2 w1 = conv1_a(wp1, lane);
    const f32x4 b1 = conv_bias(prm, P_B1, lane);
    const W2 w2a = conv2_a(wp2, lane, 0), w2b = conv2_a(wp2, lane, 16);
    const f32x4 b2a = conv_bias(prm, P_B2, lane), b2b = conv_bias(prm, P_B2 + 16, lane);
    const int mb3 = wv & 1;
    const W3 w3 = conv3_a(wp3, lane, 16 * mb3);
    const f32x4 b3 = conv_bias(prm, P_B3 + 16 * mb3, lane);
    const f32x4 hw = head_w(prm, 16 * mb3, lane);
    const float b4 = bf(prm[P_B4]);

    // lane-constant LDS byte offsets (units add compile-time strides)
    // conv1: parity wave & 1, rows from r1b; column C1 = 2 m + parity; lane
    // group g reads tap row min(g, 2)
    const int par1 = wv & 1, r1b = wv < 2 ? 0 : F_R1A;
    const int in_off = (2 * r1b + min(g, 2)) * F0S + 8 * m + 4 * par1;
    const int a1_woff = (par1 * F1H + r1b) * RS1 + (g >> 1) * 16 * F1J + 16 * m + 8 * (g & 1);
    // conv2: rows wave + 4 i; lane m is output column m (15 is the pad
    // column); chunk c, lane group g reads tap 2 c + g / 2, channel half
    // g & 1 (tap 8: channels 4 g ..)
    int a1_roff[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const int t = 2 * c + (g >> 1), ky = t / 3, kx = t % 3;
        a1_roff[c] = ((kx & 1) * F1H + 2 * wv + ky) * RS1 + (g & 1) * 16 * F1J + 16 * (m + (kx >> 1));
    }
    const int a1_roff8 = (2 * wv + 2) * RS1 + (g >> 1) * 16 * F1J + 16 * (m + 1) + 8 * (g & 1);
    // output column m: parity m & 1, pair m >> 1, channel quarter 2 mb + g / 2
    const int a2_woff = (m & 1) * P2 + wv * RS2 + (g >> 1) * 16 * F2J + 16 * (m >> 1) + 8 * (g & 1);
    // conv3: unit u3 = (wave >> 1) + 2 i covers grid rows 2 u3, 2 u3 + 1 of
    // the tile, lane m at (r3, c3) = (2 u3 + m / 8, m % 8) (c3 = 7 is not a
    // position); tap (0, 0) here, the others add constants
    int a2_roff[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const int r3 = 2 * ((wv >> 1) + 2 * i) + (m >> 3), c3 = m & 7;
        a2_roff[i] = (2 * r3) * RS2 + g * 16 * F2J + 16 * c3;
    }

    uint8_t *const a1b = (uint8_t *)s_a1;
    uint8_t *const a2b = (uint8_t *)s_a2;

    int cursor = find_image(pre_tiles, n, first);
    FTile f_prev{0, 0, 0}, f_cur = fused_tile(imgs, pre_tiles, n, tile_at(0), cursor);
    FTile f_next = K > 1 ? fused_tile(imgs, pre_tiles, n, tile_at(1), cursor) : f_cur;
    uint32_t pf[F_LD];
    {
        const CnnImg im = imgs[f_cur.img];
        fused_fetch(pyr, im, f_cur, rr, jj, pf);
        fused_stage(s_in, im, f_cur, rr, jj, pf);
    }
    if (K > 1) fused_fetch(pyr, imgs[f_next.img], f_next, rr, jj, pf);
    __syncthreads();

    for (int k = 0; k <= K; k++) {
        // phase X: conv1 of tile k (input -> conv1 planes) and conv3 + head
        // of tile k - 1 (conv2 planes -> head sums)
        if (k < K) {
            const CnnImg im = imgs[f_cur.img];
            const int Y1 = 4 * f_cur.Y3 - 3, X1 = 4 * f_cur.X3 - 3;
            const uint32_t rows = row_bits(-Y1, im.h1 - Y1) >> r1b;       // bit i: row r1b + i inside
            const bool col_ok = X1 + 2 * m + par1 >= 0 && X1 + 2 * m + par1 < im.w1;
            auto run = [&](auto masked, int i0, auto n_units) {
                constexpr int NU = decltype(n_units)::value;
                uint2 xb[NU];
#pragma unroll
                for (int j = 0; j < NU; j++) {
                    const uint8_t *src = s_in + in_off + (i0 + j) * 2 * F0S;
                    xb[j] = make_uint2(*(const uint32_t *)src, *(const uint32_t *)(src + 4));
                }
#pragma unroll
                for (int j = 0; j < NU; j++) {
                    uint2 o = relu_h4(mfma_settle(mfma16(w1, xb[j], b1)));
                    if constexpr (decltype(masked)::value) {
                        const bool ok = col_ok && ((rows >> (i0 + j)) & 1u);
                        o.x = ok ? o.x : 0u;
                        o.y = ok ? o.y : 0u;
                    }
                    *(uint2 *)(a1b + a1_woff + (i0 + j) * RS1) = o;
                }
            };
            using T6 = std::integral_constant<int, 6>;
            using T3 = std::integral_constant<int, 3>;
            const bool inside = Y1 >= 0 && Y1 + F1H <= im.h1 && X1 >= 0 && X1 + F1W <= im.w1;
            if (inside) {
                run(std::false_type{}, 0, T6{});
                run(std::false_type{}, 6, T6{});
                if (wv >= 2) run(std::false_type{}, 12, T3{});
            } else {
                run(std::true_type{}, 0, T6{});
                run(std::true_type{}, 6, T6{});
                if (wv >= 2) run(std::true_type{}, 12, T3{});
            }
        }
        if (k > 0) {
#pragma unroll
            for (int i = 0; i < 2; i++) {
                if (i == 1 && wv >= 2) break;                              // uniform
                uint4 bt[9];
#pragma unroll
                for (int t = 0; t < 9; t++) {
                    const int ky = t / 3, kx = t % 3;
                    bt[t] = *(const uint4 *)(a2b + a2_roff[i] + (kx & 1) * P2 + ky * RS2 + 16 * (kx >> 1));
                }
                // two independent chains (taps 0-4 from the bias, 5-8 from
                // zero) halve the dependent MFMA latency
                f32x4 acc = b3, acc2 = splat4(0.f);
#pragma unroll
                for (int t = 0; t < 5; t++) acc = mfma32(w3.t[t], bt[t], acc);
#pragma unroll
                for (int t = 5; t < 9; t++) acc2 = mfma32(w3.t[t], bt[t], acc2);
                const float part = head16(relu4(mfma_settle(acc) + mfma_settle(acc2)), hw);
                const int r3 = 2 * ((wv >> 1) + 2 * i) + (m >> 3), c3 = m & 7;
                if (g == 0 && c3 < F3W) s_head[mb3][r3 * F3W + c3] = part;
            }
        }
        __syncthreads();
        // phase Y: staging of tile k + 1 and the fetch of tile k + 2, logits
        // of tile k - 1, conv2 of tile k (conv1 planes -> conv2 planes)
        FTile f_new = f_next;
        if (k + 1 < K) {
            fused_stage(s_in, imgs[f_next.img], f_next, rr, jj, pf);
            if (k + 2 < K) {
                f_new = fused_tile(imgs, pre_tiles, n, tile_at(k + 2), cursor);
                fused_fetch(pyr, imgs[f_new.img], f_new, rr, jj, pf);
            }
        }
        const int zp = tid;
        if (k > 0 && zp < F_NPOS) {
            const CnnImg im = imgs[f_prev.img];
            const int gy = f_prev.Y3 + zp / F3W, gx = f_prev.X3 + zp % F3W;
            if (gy < im.h4 && gx < im.w4) z[im.px4 + (int64_t)gy * im.w4 + gx] = (s_head[0][zp] + s_head[1][zp]) + b4;
        }
        if (k < K) {
            const CnnImg im = imgs[f_cur.img];
            const int Y2 = 2 * f_cur.Y3 - 1, X2 = 2 * f_cur.X3 - 1;
            const uint32_t rows = row_bits(-Y2, im.h2 - Y2);
            const bool col_ok = X2 + m >= 0 && X2 + m < im.w2;
            const bool inside = Y2 >= 0 && Y2 + F2H <= im.h2 && X2 >= 0 && X2 + F2W <= im.w2;
            auto unit = [&](auto masked, int i) {
                B2 b;
#pragma unroll
                for (int c = 0; c < 4; c++) b.c[c] = *(const uint4 *)(a1b + a1_roff[c] + i * 8 * RS1);
                b.t8 = *(const uint2 *)(a1b + a1_roff8 + i * 8 * RS1);
                uint2 oa = relu_h4(mfma_settle(conv2_mfma(w2a, b, b2a)));
                uint2 ob = relu_h4(mfma_settle(conv2_mfma(w2b, b, b2b)));
                if constexpr (decltype(masked)::value) {
                    const bool ok = col_ok && ((rows >> (wv + 4 * i)) & 1u);
                    oa.x = ok ? oa.x : 0u;
                    oa.y = ok ? oa.y : 0u;
                    ob.x = ok ? ob.x : 0u;
                    ob.y = ok ? ob.y : 0u;
                }
                *(uint2 *)(a2b + a2_woff + i * 4 * RS2) = oa;
                *(uint2 *)(a2b + a2_woff + i * 4 * RS2 + 2 * 16 * F2J) = ob;
            };
            // rows wave + 4 i: three for every wave, a fourth (row 12) for wave 0
            if (inside) {
#pragma unroll
                for (int i = 0; i < 3; i++) unit(std::false_type{}, i);
                if (wv == 0) unit(std::false_type{}, 3);
            } else {
#pragma unroll
                for (int i = 0; i < 3; i++) unit(std::true_type{}, i);
                if (wv == 0) unit(std::true_type{}, 3);
            }
        }
        f_prev = f_cur;
        f_cur = f_next;
        f_next = f_new;
        __syncthreads();
    }
}

}  // namespace inf

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
                                    const float *__restrict__ a3, float *__restrict__ dz, float *__restrict__ lz,
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
        const float a = a3[p * 32 + co];
        g3[p * 32 + co] = a > 0.f ? d * bf(prm[P_W4 + co]) : 0.f;
    }
}

// Partial sums of the head gradients over a pixel range.
__global__ __launch_bounds__(256) void cnn_head_wgrad_kernel(int64_t total, const float *__restrict__ dz,
                                                             const float *__restrict__ a3,
                                                             float *__restrict__ part) {
    __shared__ float s_acc[256][33];
    const int64_t chunk = (total + CNN_PARTS - 1) / CNN_PARTS;
    const int64_t lo = blockIdx.x * chunk, hi = min(total, lo + chunk);
    float acc[33];
    for (int k = 0; k < 33; k++) acc[k] = 0.f;
    for (int64_t p = lo + threadIdx.x; p < hi; p += 256) {
        const float d = dz[p];
        for (int co = 0; co < 32; co++) acc[co] += d * a3[p * 32 + co];
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
                                                        const float *__restrict__ ain, const uint8_t *__restrict__ pyr,
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
                    else v = ain[(ib + (int64_t)iy * iw + ix) * CIN + ci];
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
                                                        const float *__restrict__ ain, const uint16_t *__restrict__ prm,
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
    if (ain[q * CIN + ci] > 0.f) {
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

// The proposer's device tables hold per-image prefix sums (pixels of each
// layer, MFMA tiles, fused tiles, cells) as int32: a batch whose totals
// reach 2^31 is refused (host only).
int32_t cnn_plan_check(const vsfe_batch *b) {
    if (b->info.n_levels < 4) return VSFE_OK;
    int64_t s1 = 0, s2 = 0, s4 = 0, st1 = 0, st2 = 0, st4 = 0, sc = 0, stf = 0;
    for (int i = 0; i < b->n_images; i++) {
        const ImageDev &im = b->images[i];
        const int64_t w3 = im.lv[3].w, h3 = im.lv[3].h;
        const int64_t w1 = (w3 + 1) / 2, h1 = (h3 + 1) / 2, w2 = (w1 + 1) / 2, h2 = (h1 + 1) / 2;
        const int64_t w4 = (w2 + 1) / 2, h4 = (h2 + 1) / 2;
        s1 += w1 * h1;
        s2 += w2 * h2;
        s4 += w4 * h4;
        st1 += (w1 * h1 + 15) / 16;
        st2 += (w2 * h2 + 15) / 16;
        st4 += (w4 * h4 + 15) / 16;
        sc += (int64_t)im.lv[0].ncx * im.lv[0].ncy;
        stf += ((w4 + inf::F3W - 1) / inf::F3W) * ((h4 + inf::F3H - 1) / inf::F3H);
    }
    const int64_t lim = (int64_t)1 << 31;
    // the layer arrays are also indexed as (pixel * 32 + channel) in 64 bits;
    // the counts themselves must stay below 2^31
    if (s1 >= lim || s2 >= lim || s4 >= lim || st1 >= lim || st2 >= lim || st4 >= lim || sc >= lim || stf >= lim)
        return fail(VSFE_ECAPACITY, "batch too large for the proposer's 32-bit prefix tables");
    return VSFE_OK;
}

int32_t cnn_setup(vsfe_batch *b) {
    if (b->info.n_levels < 4) return VSFE_OK;            // no level 3: the proposer is unavailable
    const int32_t rc = cnn_plan_check(b);
    if (rc) return rc;
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
        stf += (int64_t)((c.w4 + inf::F3W - 1) / inf::F3W) * ((c.h4 + inf::F3H - 1) / inf::F3H);
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
    P->off_hp1 = at;
    at = align256(at + 16 * 4 * 4 * 2);
    P->off_hp2 = at;
    at = align256(at + 32 * 9 * 16 * 2);
    P->off_hp3 = at;
    at = align256(at + 32 * 9 * 32 * 2);
    P->off_a1 = at;
    at = align256(at + s1 * 16 * 4);
    P->off_a2 = at;
    at = align256(at + s2 * 32 * 4);
    P->off_a3 = at;
    at = align256(at + s4 * 32 * 4);
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
    uint16_t *hp1 = (uint16_t *)(ws + P->off_hp1), *hp2 = (uint16_t *)(ws + P->off_hp2),
             *hp3 = (uint16_t *)(ws + P->off_hp3);
    float *a1 = (float *)(ws + P->off_a1), *a2 = (float *)(ws + P->off_a2), *a3 = (float *)(ws + P->off_a3);
    hipLaunchKernelGGL(cnn_pack_kernel, dim3((32 * 9 * 32 + 255) / 256), dim3(256), 0, st, prm, wp2, wp3, hp1, hp2,
                       hp3);
    if (P->t1 > 0)
        hipLaunchKernelGGL(tr::cnn_conv1_kernel, dim3((unsigned)((P->t1 + 3) / 4)), dim3(256), 0, st, P->d_img,
                           pre + 6 * (n + 1), n, P->t1, pyr, prm, a1);
    if (P->t2 > 0)
        hipLaunchKernelGGL(tr::cnn_conv2_kernel, dim3((unsigned)((P->t2 + 3) / 4)), dim3(256), 0, st, P->d_img,
                           pre + 3 * (n + 1), n, P->t2, a1, a2, wp2, prm);
    if (P->t4 > 0)
        hipLaunchKernelGGL(tr::cnn_conv3_kernel, dim3((unsigned)((P->t4 + 3) / 4)), dim3(256), 0, st, P->d_img,
                           pre + 4 * (n + 1), n, P->t4, a2, a3, wp3, prm, z);
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
    uint16_t *hp1 = (uint16_t *)(ws + P->off_hp1), *hp2 = (uint16_t *)(ws + P->off_hp2),
             *hp3 = (uint16_t *)(ws + P->off_hp3);
    hipLaunchKernelGGL(cnn_pack_kernel, dim3((32 * 9 * 32 + 255) / 256), dim3(256), 0, st, params_bf16, wp2, wp3,
                       hp1, hp2, hp3);
    if (P->tf > 0) {
        // persistent: a multiple of 8 blocks (one tile range per XCD), at
        // most as many as are resident at once
        static const int64_t resident = [] {
            int dev = 0, n_cu = 0, per_cu = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, inf::cnn_fused_fwd_kernel, inf::F_THREADS, 0) !=
                    hipSuccess ||
                n_cu < 1 || per_cu < 1)
                return (int64_t)256 * inf::F_BLOCKS_PER_CU;
            return (int64_t)n_cu * per_cu;
        }();
        const int64_t per_xcd = std::max<int64_t>(1, std::min(resident / N_XCD, (P->tf + N_XCD - 1) / N_XCD));
        hipLaunchKernelGGL(inf::cnn_fused_fwd_kernel, dim3((unsigned)(per_xcd * N_XCD)), dim3(inf::F_THREADS), 0, st,
                           P->d_img, P->d_pre + 7 * (P->n + 1), P->n, (int)P->tf, pyr, params_bf16, hp1, hp2, hp3,
                           grid_logits);
    }
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
    float *a1 = (float *)(ws + P->off_a1), *a2 = (float *)(ws + P->off_a2), *a3 = (float *)(ws + P->off_a3);
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
