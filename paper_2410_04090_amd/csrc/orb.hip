// ORB orientation and rBRIEF descriptors for all levels in one launch
// (Sec. III-2: Gaussian smoothing, then extraction for every scale at once).
//
// One 64-lane wave per keypoint.  The wave stages the 37 x 37 neighbourhood
// of its keypoint in LDS with 32-bit loads (coordinates clamped to the
// level, which makes the clamp-to-edge smoothing exact), each byte stored
// as p - 128 (a signed byte), then:
//  * intensity centroid over the disc u^2 + v^2 <= 225 of the unsmoothed
//    level, one lane per disc row: S_v = sum_u I and T_v = sum_u (u+16) I as
//    signed dot products of 4 bytes against constant weight words
//    (v_dot4_i32_i8) plus the per-row constants that undo the -128;
//    m10 = sum_v (T_v - 16 S_v), m01 = sum_v v S_v, reduced on the DPP network;
//  * orientation bin: 30 lanes compare m with the Q14 bin boundaries at
//    6 + 12 j degrees by exact integer half-plane / cross-product tests,
//    a ballot counts them (bin = count mod 30, 0 for m = 0);
//  * smoothing only of the 31 x 31 patch the tests can touch, separable
//    7-tap [18 33 49 56 49 33 18] / 256 with each pass rounded half up;
//    both passes are exact integer products with a banded weight matrix on
//    v_mfma_i32_16x16x32_i8 over the signed bytes.  The accumulators start
//    at the rounding constant, so byte 1 of each one is the rounded result:
//    the horizontal pass starts at 128 and yields H - 128 directly as the
//    signed input of the vertical pass, which starts at 128 * 256 + 128 and
//    yields the unsigned result; four results pack into a word with two
//    v_perm.  The horizontal pass writes its result transposed so the
//    vertical pass reads 8 rows of one column per lane, and the final patch
//    is stored transposed;
//  * 256 tests on the bin-rotated pattern (per bin, precomputed in the
//    context as byte offsets into the stored patch), 64 per ballot, written
//    as 8 words.
// The whole-level smoothed pyramid never touches HBM.
#include <string.h>

#include <algorithm>

#include "vsfe_internal.h"

namespace vsfe {

constexpr int ORB_WAVES = 4;
constexpr int R_STRIDE = 40;      // staged 37 x 37 neighbourhood, one row per 40 bytes (10 words)
constexpr int R_BYTES = 48 * R_STRIDE + 32;   // 48 rows (3 MFMA row tiles) + read slack
constexpr int HT_STRIDE = 56;     // horizontal pass, transposed: [column][row], 37 of 48 rows used (14 words: columns spread over the banks)
constexpr int HT_BYTES = 32 * HT_STRIDE + 16;
constexpr int B_STRIDE = ORB_PATCH_STRIDE;   // final smoothed patch, transposed: [column][row], 31 used
constexpr int B_BYTES = 32 * B_STRIDE;
constexpr uint32_t W_LO = 18u | (33u << 8) | (49u << 16) | (56u << 24);
constexpr uint32_t W_HI = 49u | (33u << 8) | (18u << 16);

struct OrbArgs {
    OrbTables tab;
    int n_max, n_images, blur, aligned0;
};

// Per disc row v = -15..15: byte u' (u = u' - 15) of 8 words is 0xff inside
// the disc u^2 + v^2 <= 225, 0 elsewhere (and at u' = 31).  A row's masked
// bytes dotted with 1 give S_v, dotted with the ramp u' + 1 = u + 16 (the
// same for every row: bytes 4k + 1 .. 4k + 4 of word k) give T_v.
struct DiscTables {
    uint32_t mask[31][8];
};
__constant__ DiscTables c_disc;

__host__ __device__ constexpr uint32_t ramp_word(int k) {
    return (uint32_t)(4 * k + 1) | ((uint32_t)(4 * k + 2) << 8) | ((uint32_t)(4 * k + 3) << 16) |
           ((uint32_t)(4 * k + 4) << 24);
}

// Constant MFMA operand of the smoothing (v_mfma_i32_16x16x32_i8, 8 bytes per
// lane: lane l covers K = 8 (l / 16) .. + 7 of row / column l % 16): the band
// W[k][n] = w[k - n], zero outside 0 <= k - n <= 6.  A 16-wide output tile
// starting at index 16 t reads inputs 16 t .. 16 t + 21, so one K chunk of 32
// starting at 16 t covers it, and relative to that start the band is the same
// for every tile: it is B of the horizontal pass (K = input column, n =
// output column) and A of the vertical pass (K = input row, n = output row).
struct SmoothTables {
    uint64_t band[64];
};
__constant__ SmoothTables c_smooth;

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Each wave works on its own keypoint and its own LDS region, so the waves
// of a block never wait for one another: a wave's LDS operations complete
// in order, and this fence keeps the compiler from moving reads up.
__device__ __forceinline__ void wave_lds_fence() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int half_plane(int64_t x, int64_t y) { return (y < 0 || (y == 0 && x < 0)) ? 1 : 0; }

__device__ __forceinline__ uint32_t fetch4c(const uint8_t *row, int x, int w) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) v |= (uint32_t)row[min(max(x + j, 0), w - 1)] << (8 * j);
    return v;
}

// Sum over lanes 0..31 on the DPP network (row shifts, then row 0's last
// lane broadcast into row 1); valid in lane 31.
__device__ __forceinline__ int sum_lanes32(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    return __builtin_amdgcn_readlane(v, 31);
}

// Byte 1 of four accumulators, packed into one word.
__device__ __forceinline__ uint32_t pack_byte1(const i32x4 &a) {
    return __builtin_amdgcn_perm((uint32_t)a[1], (uint32_t)a[0], 0x0C0C0501u) |
           __builtin_amdgcn_perm((uint32_t)a[3], (uint32_t)a[2], 0x05010C0Cu);
}

// Persistent waves: a wave takes keypoint slots first, first + W, ... (W =
// waves in the grid) and loads the next keypoint's neighbourhood into
// registers while it computes the current one.  The per-lane constant
// tables are read once, and the current keypoint's pattern is read before
// the next prefetch is issued, so no wait inside the loop waits for the
// prefetch.  Slot state is wave-uniform (scalar registers).
// At most 80 VGPRs, six waves per SIMD (the LDS of six blocks fits): the
// only spills are on the clamped-border staging path and the unsmoothed
// path; seven waves (72 VGPRs) spill in the loop and run slower.
__global__ __launch_bounds__(256, 6) void orb_kernel(const ImageDev *__restrict__ imgs, const uint8_t *__restrict__ images,
                                                  const uint8_t *__restrict__ pyr, vsfe_kp_soa kps,
                                                  const int32_t *__restrict__ kp_count,
                                                  const uint32_t *__restrict__ pat_off, uint32_t *__restrict__ desc,
                                                  OrbArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t s_r[ORB_WAVES][R_BYTES / 4];
    __shared__ __attribute__((aligned(16))) uint32_t s_ht[ORB_WAVES][HT_BYTES / 4];
    __shared__ __attribute__((aligned(16))) uint32_t s_b[ORB_WAVES][B_BYTES / 4];
    __shared__ __attribute__((aligned(16))) uint32_t s_disc[31 * 8];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int mrow = lane & 15, grp = lane >> 4;
    uint8_t *R = (uint8_t *)s_r[wave];
    uint8_t *HT = (uint8_t *)s_ht[wave];
    uint8_t *BT = (uint8_t *)s_b[wave];

    // disc masks in LDS (read per keypoint, not held in registers); cS / cT
    // undo the -128 of the staged bytes
    for (int k = threadIdx.x; k < 31 * 8; k += 256) s_disc[k] = (&c_disc.mask[0][0])[k];
    int cS = 0, cT = 0;
    if (lane < 31) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            cS += (int)__builtin_amdgcn_udot4(c_disc.mask[lane][k] & 0x01010101u, 0x80808080u, 0u, false);
            cT += (int)__builtin_amdgcn_udot4(c_disc.mask[lane][k] & ramp_word(k), 0x80808080u, 0u, false);
        }
    }
    __syncthreads();
    const long band = (long)c_smooth.band[lane];
    int bx = 0, by = 0;                          // Q14 boundary directions (32-bit: fewer registers)
    if (lane < 30) {
        bx = a.tab.bin_x[lane];
        by = a.tab.bin_y[lane];
    }
    // staging tasks of this lane: dword t = lane + 64 u is row t / 10, word t % 10
    // (its LDS word is t itself: rows are 10 words apart)
    static_assert(R_STRIDE == 40, "staging assumes 10 words per row");
    // (rows < 64: one byte each, two registers instead of six)
    uint32_t t_rows[2] = {0u, 0u};
#pragma unroll
    for (int u = 0; u < 6; u++) t_rows[u >> 2] |= (uint32_t)((lane + 64 * u) / 10) << (8 * (u & 3));
    auto t_row = [&](int u) { return (int)((t_rows[u >> 2] >> (8 * (u & 3))) & 0xFFu); };

    // Keypoint metadata of the wave's next 64 iterations, one iteration per
    // lane (slot, counts, coordinates, level geometry: three dependent
    // memory round trips paid once per 64 keypoints instead of once per
    // keypoint); an iteration reads its lane's values with readlane.
    const int64_t first = (int64_t)xcd_item(blockIdx.x, gridDim.x) * ORB_WAVES + wave;
    const int64_t nw = (int64_t)gridDim.x * ORB_WAVES;
    const int64_t n_slots = (int64_t)a.n_images * a.n_max;
    // flags: 1 = active, 2 = level 0, 4 = interior (the whole 40 x 37 window
    // inside an aligned level with a pitch below 2^24), bits 8-9 = the
    // window's byte offset in its first word; m_addr = the window's first
    // word (interior) or the level's first byte
    uint32_t m_xy = 0, m_wh = 0, m_pitch = 0, m_flags = 0;
    uint64_t m_addr = 0;
    auto load_meta = [&](int64_t k0) {
        const int64_t sl = first + (k0 + lane) * nw;
        m_flags = 0;
        if (sl < n_slots) {
            const int image = (int)sl / a.n_max, i = (int)sl - image * a.n_max;
            if (i < kp_count[image]) {
                const int x = kps.x[sl], y = kps.y[sl], lvl = kps.level[sl];
                const LevelDev &lv = imgs[image].lv[lvl];
                m_xy = (uint32_t)x | ((uint32_t)y << 16);
                m_wh = (uint32_t)lv.w | ((uint32_t)lv.h << 16);
                m_pitch = (uint32_t)lv.pitch;
                const uint8_t *src = (lvl == 0 ? images : pyr) + lv.offset;
                const int xs = (x - 18) & ~3;
                const bool aligned = lvl != 0 || a.aligned0;
                const bool interior = aligned && y >= 18 && y + 18 < lv.h && xs >= 0 && xs + 40 <= lv.w &&
                                      lv.pitch < (1 << 24);
                m_addr = (uint64_t)(interior ? src + (int64_t)(y - 18) * lv.pitch + xs : src);
                m_flags = 1u | (lvl == 0 ? 2u : 0u) | (interior ? 4u : 0u) | ((uint32_t)((x - 18) - xs) << 8);
            }
        }
    };

    // prefetched state of the next keypoint (iteration j of the metadata batch)
    bool p_act = false;
    int p_delta = 0;
    uint32_t p_v[6];
    auto fetch = [&](int j) {
        const uint32_t fl = __builtin_amdgcn_readlane(m_flags, j);
        p_act = (fl & 1u) != 0;
        if (!p_act) return;
        p_delta = (int)((fl >> 8) & 3u);
        const int pitch = (int)__builtin_amdgcn_readlane(m_pitch, j);
        // (a global-memory pointer: rebuilt from an integer it would be a
        // generic one, read with flat loads.  readlane returns a signed int:
        // both halves go through uint32_t, or a low half with bit 31 set
        // would be sign-extended into the high half)
        typedef const __attribute__((address_space(1))) uint8_t gbyte;
        const uint32_t a_hi = (uint32_t)__builtin_amdgcn_readlane((uint32_t)(m_addr >> 32), j);
        const uint32_t a_lo = (uint32_t)__builtin_amdgcn_readlane((uint32_t)m_addr, j);
        gbyte *addr = (gbyte *)(((uint64_t)a_hi << 32) | a_lo);
        if (fl & 4u) {
            // the whole window lies inside the level: plain 32-bit loads at
            // 32-bit per-lane offsets from the uniform window address
            // (24-bit multiply-adds, scalar-base addressing; 36 rows of a
            // pitch below 2^24 stay below 2^32)
            const uint32_t step = (uint32_t)(pitch - 40);
#pragma unroll
            for (int u = 0; u < 6; u++) {
                const uint32_t off = __umul24((uint32_t)t_row(u), step) + 4u * (uint32_t)(lane + 64 * u);
                p_v[u] = (lane + 64 * u < 37 * 10) ? *(const __attribute__((address_space(1))) uint32_t *)(addr + off) : 0u;
            }
        } else {
            const uint32_t xy = __builtin_amdgcn_readlane(m_xy, j), wh = __builtin_amdgcn_readlane(m_wh, j);
            const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
            const int lw = (int)(wh & 0xFFFFu), lh = (int)(wh >> 16);
            const int xs = (x - 18) & ~3;
#pragma unroll
            for (int u = 0; u < 6; u++) {
                p_v[u] = 0u;
                if (lane + 64 * u < 37 * 10) {
                    const int gy = min(max(y - 18 + t_row(u), 0), lh - 1);
                    p_v[u] = fetch4c((const uint8_t *)(addr + (int64_t)gy * pitch), xs + 4 * (lane + 64 * u - 10 * t_row(u)), lw);
                }
            }
        }
    };

    load_meta(0);
    fetch(0);
    // (the slot advances by nw per iteration: an add, not a 64-bit multiply)
    int64_t slot = first;
    for (int64_t k = 0; slot < n_slots; k++, slot += nw) {
        const bool active = p_act;
        const int delta = p_delta;
        if (active) {
#pragma unroll
            for (int u = 0; u < 6; u++)
                if (lane + 64 * u < 37 * 10) s_r[wave][lane + 64 * u] = p_v[u] ^ 0x80808080u;
        }
        wave_lds_fence();

        // intensity centroid: lane v' = v + 15 < 31 sums its disc row
        int m10 = 0, m01 = 0;
        if (active && lane < 31) {
            const int al = (delta + 3) & 3;
            const uint32_t *w = (const uint32_t *)(R + (lane + 3) * R_STRIDE + ((delta + 3) & ~3));
            int S = cS, T = cT;
            uint32_t prev = w[0];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const uint32_t nxt = w[k + 1];
                const uint32_t b4 = __builtin_amdgcn_alignbyte(nxt, prev, al);
                const int xm = (int)(b4 & s_disc[lane * 8 + k]);
                S = __builtin_amdgcn_sdot4(xm, 0x01010101, S, false);
                T = __builtin_amdgcn_sdot4(xm, (int)ramp_word(k), T, false);
                prev = nxt;
            }
            m10 = T - 16 * S;
            m01 = (lane - 15) * S;
        }
        m10 = sum_lanes32(m10);
        m01 = sum_lanes32(m01);
        // orientation bin: lane j < 30 tests angle(m) >= angle(boundary j)
        bool ge = false;
        if (lane < 30) {
            const int hm = half_plane(m10, m01), hb = half_plane(bx, by);
            ge = hm != hb ? hm > hb : ((int64_t)bx * m01 - (int64_t)by * m10 >= 0);
        }
        const uint64_t gem = __ballot(ge);
        const int bin = (m10 == 0 && m01 == 0) ? 0 : (__popcll(gem) % 30);
        // this keypoint's rotated pattern, then the next keypoint's rows
        uint32_t qv[4];
        if (active) {
            const uint32_t *pr = pat_off + bin * 256;
#pragma unroll
            for (int rnd = 0; rnd < 4; rnd++) qv[rnd] = pr[rnd * 64 + lane];
        }
        const int jn = (int)((k + 1) & 63);
        if (jn == 0) load_meta(k + 1);
        fetch(jn);

        if (active) {
            if (a.blur) {
                // horizontal pass on MFMA: H[r][c] - 128 = (128 + sum_j R'[r][j] W[j][c]) >> 8
                // with R'[r][j] = R[r][j + delta] - 128; 3 row tiles x 2 column
                // tiles, one K chunk each (inputs 16 nt .. 16 nt + 31; the band
                // is zero beyond 16 nt + 21, which also covers the bytes read
                // past a row's end).  Written transposed, 4 rows per dword.
#pragma unroll
                for (int mt = 0; mt < 3; mt++) {
#pragma unroll
                    for (int nt = 0; nt < 2; nt++) {
                        const uint32_t *w = (const uint32_t *)(R + (16 * mt + mrow) * R_STRIDE + 16 * nt + 8 * grp);
                        const uint32_t d0 = w[0], d1 = w[1], d2 = w[2];
                        const uint32_t lo = __builtin_amdgcn_alignbyte(d1, d0, delta);
                        const uint32_t hi = __builtin_amdgcn_alignbyte(d2, d1, delta);
                        const long av = (long)(((uint64_t)hi << 32) | lo);
                        const i32x4 acc = __builtin_amdgcn_mfma_i32_16x16x32_i8(av, band, i32x4{128, 128, 128, 128}, 0, 0, 0);
                        *(uint32_t *)(HT + (16 * nt + mrow) * HT_STRIDE + 16 * mt + 4 * grp) = pack_byte1(mfma_settle(acc));
                    }
                }
                wave_lds_fence();
                // vertical pass on MFMA: V[r'][c] = (32896 + sum_r W[r][r'] (H[r][c] - 128)) >> 8,
                // 2 row tiles x 2 column tiles, one K chunk each (rows 16 mt ..
                // 16 mt + 31), B read from the transposed H (8 rows of one
                // column per lane); the output is written transposed, 4 rows per dword
#pragma unroll
                for (int mt = 0; mt < 2; mt++) {
#pragma unroll
                    for (int nt = 0; nt < 2; nt++) {
                        const uint2 hv = *(const uint2 *)(HT + (16 * nt + mrow) * HT_STRIDE + 16 * mt + 8 * grp);
                        const long bv = (long)((((uint64_t)hv.y) << 32) | hv.x);
                        const i32x4 acc =
                            __builtin_amdgcn_mfma_i32_16x16x32_i8(band, bv, i32x4{32896, 32896, 32896, 32896}, 0, 0, 0);
                        s_b[wave][((16 * nt + mrow) * B_STRIDE + 16 * mt + 4 * grp) >> 2] = pack_byte1(mfma_settle(acc));
                    }
                }
            } else {
                for (int t = lane; t < 31 * 31; t += 64) {
                    const int c = t / 31, r = t - c * 31;
                    BT[c * B_STRIDE + r] = R[(r + 3) * R_STRIDE + delta + c + 3] ^ 0x80u;
                }
            }
        }
        wave_lds_fence();
        if (active) {
            uint32_t words[8];
#pragma unroll
            for (int rnd = 0; rnd < 4; rnd++) {
                const int pa = BT[qv[rnd] & 0xFFFFu];
                const int pb = BT[qv[rnd] >> 16];
                const uint64_t bits = __ballot(pa < pb);
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
        wave_lds_fence();
    }
}

static bool g_disc_ready[64];

static int32_t upload_disc(int device, hipStream_t st) {
    if (device >= 0 && device < 64 && g_disc_ready[device]) return VSFE_OK;
    DiscTables t;
    memset(&t, 0, sizeof(t));
    for (int vi = 0; vi < 31; vi++) {
        const int v = vi - 15;
        for (int ui = 0; ui < 31; ui++) {
            const int u = ui - 15;
            if (u * u + v * v > 225) continue;
            t.mask[vi][ui >> 2] |= 0xFFu << (8 * (ui & 3));
        }
    }
    (void)st;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_disc), &t, sizeof(t), 0, hipMemcpyHostToDevice) != hipSuccess)
        return fail(VSFE_EHIP, "upload of the disc tables failed");
    static const int kw[7] = {18, 33, 49, 56, 49, 33, 18};
    SmoothTables sm;
    memset(&sm, 0, sizeof(sm));
    for (int l = 0; l < 64; l++) {
        uint64_t band = 0;
        for (int bb = 0; bb < 8; bb++) {
            const int d = 8 * (l >> 4) + bb - (l & 15);          // k - n
            if (d >= 0 && d <= 6) band |= (uint64_t)kw[d] << (8 * bb);
        }
        sm.band[l] = band;
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_smooth), &sm, sizeof(sm), 0, hipMemcpyHostToDevice) != hipSuccess)
        return fail(VSFE_EHIP, "upload of the smoothing tables failed");
    if (device >= 0 && device < 64) g_disc_ready[device] = true;
    return VSFE_OK;
}

int32_t orb_prepare(int device) { return upload_disc(device, nullptr); }

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
    a.aligned0 = b->aligned_input && (((uintptr_t)images & 3) == 0) ? 1 : 0;
    const int64_t slots = b->info.kp_capacity;
    if (slots >= ((int64_t)1 << 31)) return fail(VSFE_ECAPACITY, "more than 2^31 keypoint slots");
    int64_t blocks = (slots + ORB_WAVES - 1) / ORB_WAVES;
    if (blocks <= 0) return VSFE_OK;
    static const int64_t resident = [] {
        int dev = 0, n_cu = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, orb_kernel, 256, 0) != hipSuccess || n_cu < 1 ||
            per_cu < 1)
            return (int64_t)2048;
        return (int64_t)n_cu * per_cu;
    }();
    blocks = std::min(blocks, resident);
    hipLaunchKernelGGL(orb_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, b->d_images, images, pyr,
                       *kps, kp_count, ctx->d_pattern_off, desc, a);
    return check_launch("orb_describe");
}
