// FAST with Bounded Rectification, corner response and Feature Culling,
// fused in one launch over every (image, level, cell tile).
//
//  * Labels (Sec. II-A, Eq. 1): bright if I_p > I_c + eps, dark if
//    I_p < I_c - eps, on the 16-pixel radius-3 ring; |I_p - I_c| = eps is
//    similar.
//  * Corner (Eq. 3): the longest cyclic bright or dark run N satisfies
//    p_min <= N <= p_max (p_max = 16 is plain FAST, Eq. 2).
//  * Response (Sec. III-1): sum over the ring of |I_c - I_p|.
//  * Feature Culling (Sec. II-C-1): per cell the largest key
//    (score << 10) | (1023 - offset in cell), i.e. the strongest corner and,
//    on ties, the first in raster order; a cell without an eps_hi corner
//    takes its best eps_lo corner and is flagged.
//
// GPU mapping (one 256-thread block per rectangle of whole cells, at most
// 128 x 32 pixels):
//  1. Stage the tile and a 3-pixel halo in LDS in a split-half layout: the
//     32-bit word at (row, col) holds pixel col of the left 64-pixel half in
//     its low 16 bits and pixel col + 64 in its high 16 bits, so any ring
//     offset of a lane's two pixels is one aligned 32-bit LDS read.  Rows
//     are fetched as 32-bit words and split with v_perm.
//  2. Prefilter every pixel pair with packed 16-bit min / max / saturating
//     subtract: a cyclic run of >= 9 ring pixels covers two adjacent compass
//     pixels (0, 4, 8, 12), i.e. one of {0, 8} and one of {4, 12}, so a
//     bright run needs min(max(p0, p8), max(p4, p12)) > c + eps (dark:
//     max(min(p0, p8), min(p4, p12)) < c - eps), at the weaker threshold.
//  3. Candidates go to per-wave LDS queues (ballot prefix), so the full ring
//     test runs densely over candidates only: masks are built with alignbit
//     (one op inserts one sign bit; run lengths do not depend on bit order)
//     and runs are tested by shift-and doubling.
//  4. Keys reduce per cell with LDS atomicMax (order independent, so the
//     result is exact and deterministic) and are written once per cell.
#include "vsfe_internal.h"

namespace vsfe {

constexpr int FT_HALF = 64;                      // lanes per row; lane owns cols l and l + 64
constexpr int FT_CHUNKS = 6;                     // 16-byte source chunks per row and half
// LDS words per row: 70 used + 16-byte alignment slack; 100 = 36 mod 64, so
// the rows of a 7 x 7 window (and rows 4 apart) fall in different banks
constexpr int FT_W = 100;
constexpr int FT_MAX_ROWS = 32;
constexpr int FT_ROWS = FT_MAX_ROWS + 6;
constexpr int FT_MAX_CELLS = 512;
constexpr int FT_QSEG = (FT_MAX_ROWS / 4) * 2 * FT_HALF + FT_HALF;   // + one dummy slot per lane
constexpr int FT_Q2 = 2048;                      // second-stage queue (overflow handled inline)

struct DetParams {
    int eps_hi, eps_lo, p_min, p_max, border, eps_min, aligned;
};

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ us2 as_us2(uint32_t v) { return __builtin_bit_cast(us2, v); }
__device__ __forceinline__ uint32_t as_u32(us2 v) { return __builtin_bit_cast(uint32_t, v); }

// ring offsets (dx, dy) in cyclic order
__constant__ int8_t c_ring_dx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
__constant__ int8_t c_ring_dy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

// Does the 16-bit mask hold a cyclic run of >= k ones (1 <= k <= 16)?  The
// mask is doubled to 32 bits so cyclic runs are contiguous; r_p marks starts
// of p-runs and k is assembled from its binary digits (k is uniform, so the
// branches are scalar).
template <bool P9>
__device__ __forceinline__ bool run_ge(uint32_t m, int k) {
    if (P9) k = 9;                               // paper setting: P_min = 9, P_max = 13
    const uint32_t r1 = m | (m << 16);
    const uint32_t r2 = r1 & (r1 >> 1);
    const uint32_t r4 = r2 & (r2 >> 2);
    const uint32_t r8 = r4 & (r4 >> 4);
    uint32_t acc = 0xFFFFFFFFu;
    int s = 0;
    if (k & 16) {
        acc &= r8 & (r8 >> 8);
        s += 16;
    }
    if (k & 8) {
        acc &= r8 >> s;
        s += 8;
    }
    if (k & 4) {
        acc &= r4 >> s;
        s += 4;
    }
    if (k & 2) {
        acc &= r2 >> s;
        s += 2;
    }
    if (k & 1) acc &= r1 >> s;
    return acc != 0;
}

template <bool P9>
__device__ __forceinline__ bool br_corner(uint32_t m, int p_min, int p_max) {
    if (P9) return run_ge<true>(m, 9) && !run_ge<false>(m, 14);
    return run_ge<false>(m, p_min) && (p_max >= 16 || !run_ge<false>(m, p_max + 1));
}

// Does level-l cell (cx, cy) overlap a kept level-0 cell?  Footprint at the
// native scale: [x S >> 16, ceil((x + c) S / 2^16)) with x = cx c, same in y.
__device__ __forceinline__ bool cell_runs(const uint8_t *mask0, const LevelDev &l0, const LevelDev &lv,
                                          int cx, int cy) {
    const int64_t S = lv.scale_q16, c = lv.cell, c0 = l0.cell;
    const int64_t fx0 = ((int64_t)cx * c * S) >> 16, fx1 = (((int64_t)cx * c + c) * S + 65535) >> 16;
    const int64_t fy0 = ((int64_t)cy * c * S) >> 16, fy1 = (((int64_t)cy * c + c) * S + 65535) >> 16;
    int a0 = (int)(fx0 / c0), a1 = (int)((fx1 - 1) / c0), b0 = (int)(fy0 / c0), b1 = (int)((fy1 - 1) / c0);
    a1 = a1 < l0.ncx - 1 ? a1 : l0.ncx - 1;
    b1 = b1 < l0.ncy - 1 ? b1 : l0.ncy - 1;
    for (int y = b0; y <= b1; y++)
        for (int x = a0; x <= a1; x++)
            if (mask0[y * l0.ncx + x]) return true;
    return false;
}

// 16 consecutive bytes of a row starting at x (zero outside [0, w)).
__device__ __forceinline__ uint4 fetch16(const uint8_t *row, int x, int w, bool aligned) {
    if (aligned && x >= 0 && x + 15 < w) return *(const uint4 *)(row + x);
    uint32_t v[4] = {0, 0, 0, 0};
    for (int j = 0; j < 16; j++)
        if (x + j >= 0 && x + j < w) v[j >> 2] |= (uint32_t)row[x + j] << (8 * (j & 3));
    return make_uint4(v[0], v[1], v[2], v[3]);
}

// Ring mask at threshold e for one polarity, bit order reversed (run
// lengths do not depend on it).  Bright: p > c + e  <=>  (c + e) - p < 0;
// dark: p < c - e  <=>  p - (c - e) < 0.  Both are (p ^ s) + t with
// (s, t) = (-1, c + e + 1) or (0, e - c), one v_xad per ring pixel.
__device__ __forceinline__ uint32_t ring_mask(const int *p, int ctr, int e, bool dark) {
    const int s = dark ? 0 : -1;
    const int t = dark ? e - ctr : ctr + e + 1;
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 16; j++) m = __builtin_amdgcn_alignbit(m, (uint32_t)((p[j] ^ s) + t), 31);
    return m;
}

template <int PF, bool LO, bool P9>
__global__ __launch_bounds__(256) void fast_br_kernel(const ImageDev *__restrict__ imgs,
                                                      const DetItem *__restrict__ items,
                                                      const uint8_t *__restrict__ images,
                                                      const uint8_t *__restrict__ pyr,
                                                      const uint8_t *__restrict__ mask,
                                                      uint32_t *__restrict__ cell_keys,
                                                      uint16_t *__restrict__ crf, DetParams prm) {
    __shared__ __attribute__((aligned(16))) uint32_t tile[FT_ROWS * FT_W];
    __shared__ uint16_t s_q[4 * FT_QSEG];
    __shared__ uint16_t s_q2[FT_Q2];
    __shared__ uint32_t s_hi[FT_MAX_CELLS], s_lo[FT_MAX_CELLS];
    __shared__ uint8_t s_run[FT_MAX_CELLS];
    __shared__ int s_qcnt[4];
    __shared__ int s_any, s_n2;

    const DetItem it = items[blockIdx.x];
    const ImageDev &im = imgs[it.image];
    const LevelDev lv = im.lv[it.level];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lv.cell;
    const int nk = it.nkx * it.nky;
    const int x0 = it.cx0 * c, y0 = it.cy0 * c;
    const int x1 = min(x0 + it.nkx * c, lv.w), y1 = min(y0 + it.nky * c, lv.h);
    const int tw = x1 - x0, th = y1 - y0;

    // learned gating: which cells of this tile run at all
    if (tid == 0) {
        s_any = 0;
        s_n2 = 0;
    }
    __syncthreads();
    for (int k = tid; k < nk; k += 256) {
        bool run = true;
        if (mask) run = cell_runs(mask + im.cell0_offset, im.lv[0], lv, it.cx0 + k % it.nkx, it.cy0 + k / it.nkx);
        s_run[k] = run;
        s_hi[k] = 0;
        s_lo[k] = 0;
        if (run) s_any = 1;
    }
    __syncthreads();
    if (!s_any && !crf) {
        for (int k = tid; k < nk; k += 256)
            cell_keys[lv.cell_offset + (int64_t)(it.cy0 + k / it.nkx) * lv.ncx + (it.cx0 + k % it.nkx)] = 0;
        return;
    }

    // 1. stage rows y0-3 .. y1+2; word column j holds image columns xb + j and
    //    xb + 64 + j.  One task = one 16-byte chunk of both halves of a row, so
    //    every thread has its two loads in flight at once.
    const uint8_t *src = (it.level == 0 ? images : pyr) + lv.offset;
    const int xb = (x0 - 3) & ~15, delta = (x0 - 3) - xb;
    const bool aligned = it.level > 0 || prm.aligned != 0;
    if (tid < (th + 6) * FT_CHUNKS) {
        const int rr = tid / FT_CHUNKS, m = tid - rr * FT_CHUNKS;
        const int gy = y0 - 3 + rr;
        uint4 L = make_uint4(0, 0, 0, 0), R = make_uint4(0, 0, 0, 0);
        if (gy >= 0 && gy < lv.h) {
            const uint8_t *row = src + (int64_t)gy * lv.pitch;
            L = fetch16(row, xb + 16 * m, lv.w, aligned);
            R = fetch16(row, xb + FT_HALF + 16 * m, lv.w, aligned);
        }
        uint4 *dst = (uint4 *)&tile[rr * FT_W + 16 * m];
        const uint32_t l4[4] = {L.x, L.y, L.z, L.w}, r4[4] = {R.x, R.y, R.z, R.w};
#pragma unroll
        for (int k = 0; k < 4; k++) {
            uint4 v;
            v.x = __builtin_amdgcn_perm(r4[k], l4[k], 0x0C040C00u);
            v.y = __builtin_amdgcn_perm(r4[k], l4[k], 0x0C050C01u);
            v.z = __builtin_amdgcn_perm(r4[k], l4[k], 0x0C060C02u);
            v.w = __builtin_amdgcn_perm(r4[k], l4[k], 0x0C070C03u);
            dst[k] = v;
        }
    }
    __syncthreads();

    // 2. prefilter, 3a. per-wave candidate queues
    //    entry = dark << 14 | bright << 13 | row << 7 | column
    const int B = prm.border;
    const int gxl = x0 + lane, gxh = x0 + FT_HALF + lane;
    const bool okl = lane < tw && gxl >= B && gxl < lv.w - B;
    const bool okh = FT_HALF + lane < tw && gxh >= B && gxh < lv.w - B;
    const uint32_t vmask = (okl ? 0xFFFFu : 0u) | (okh ? 0xFFFF0000u : 0u);
    const us2 e2 = {(unsigned short)prm.eps_min, (unsigned short)prm.eps_min};
    uint16_t *q = s_q + wave * FT_QSEG;
    const int dummy = FT_QSEG - FT_HALF + lane;
    int qn = 0;
    const int ylo = max(B - y0, 0), yhi = min(lv.h - B - y0, th);
    for (int r = wave + ((ylo - wave + 3) & ~3); r < yhi; r += 4) {
        const uint32_t *t = &tile[(r + 3) * FT_W + lane + 3 + delta];
        uint32_t tbu = vmask, tdu = vmask;
        if (PF) {
            const us2 C = as_us2(t[0]);
            const us2 P0 = as_us2(t[-3 * FT_W]), P8 = as_us2(t[3 * FT_W]);
            const us2 P4 = as_us2(t[3]), P12 = as_us2(t[-3]);
            us2 Mb, Md;
            if (PF == 2) {
                Mb = __builtin_elementwise_min(__builtin_elementwise_max(P0, P8), __builtin_elementwise_max(P4, P12));
                Md = __builtin_elementwise_max(__builtin_elementwise_min(P0, P8), __builtin_elementwise_min(P4, P12));
            } else {
                Mb = __builtin_elementwise_max(__builtin_elementwise_max(P0, P8), __builtin_elementwise_max(P4, P12));
                Md = __builtin_elementwise_min(__builtin_elementwise_min(P0, P8), __builtin_elementwise_min(P4, P12));
            }
            tbu &= as_u32(__builtin_elementwise_sub_sat(Mb, C + e2));
            tdu &= as_u32(__builtin_elementwise_sub_sat(__builtin_elementwise_sub_sat(C, e2), Md));
        }
        const uint32_t pol_l = ((tbu & 0xFFFFu) ? (1u << 13) : 0u) | ((tdu & 0xFFFFu) ? (1u << 14) : 0u);
        const uint32_t pol_h = ((tbu >> 16) ? (1u << 13) : 0u) | ((tdu >> 16) ? (1u << 14) : 0u);
        const bool cl = pol_l != 0, ch = pol_h != 0;
        const uint64_t bl = __ballot(cl), bh = __ballot(ch);
        const int nl = __popcll(bl);
        const int pl = __builtin_amdgcn_mbcnt_hi((uint32_t)(bl >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bl, 0));
        const int ph = __builtin_amdgcn_mbcnt_hi((uint32_t)(bh >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bh, 0));
        q[cl ? qn + pl : dummy] = (uint16_t)(pol_l | (r << 7) | lane);
        q[ch ? qn + nl + ph : dummy] = (uint16_t)(pol_h | (r << 7) | (FT_HALF + lane));
        qn += nl + __popcll(bh);
    }
    if (lane == 0) s_qcnt[wave] = qn;
    __syncthreads();

    const uint16_t *t16 = (const uint16_t *)tile;
    // the 16 ring pixels and the centre of tile pixel (r, col), from LDS
    auto load_ring = [&](int r, int col, int *p) {
        const uint16_t *win = t16 + 2 * (r * FT_W + (col & 63) + delta) + (col >> 6);
#pragma unroll
        for (int j = 0; j < 16; j++) p[j] = win[2 * ((c_ring_dy[j] + 3) * FT_W + c_ring_dx[j] + 3)];
        return (int)win[2 * (3 * FT_W + 3)];
    };
    // decision for a screened pixel: rb / rd = polarities with a run >= p_min at eps_min
    auto finish = [&](int r, int col, bool rb, bool rd) {
        int p[16];
        const int ctr = load_ring(r, col, p);
        bool c_hi = false, c_lo = false;
        if constexpr (P9) {
            // p_min = 9: a bright and a dark run cannot coexist, one polarity decides
            const bool dk = !rb;
            if (LO) {
                c_lo = br_corner<true>(ring_mask(p, ctr, prm.eps_lo, dk), 9, 13);
                c_hi = br_corner<true>(ring_mask(p, ctr, prm.eps_hi, dk), 9, 13);
            } else {
                c_hi = br_corner<true>(ring_mask(p, ctr, prm.eps_hi, dk), 9, 13);
            }
        } else {
            if (LO) {
                if (rb) c_lo = br_corner<false>(ring_mask(p, ctr, prm.eps_lo, false), prm.p_min, prm.p_max);
                if (rd) c_lo = c_lo || br_corner<false>(ring_mask(p, ctr, prm.eps_lo, true), prm.p_min, prm.p_max);
            }
            if (rb) c_hi = br_corner<false>(ring_mask(p, ctr, prm.eps_hi, false), prm.p_min, prm.p_max);
            if (rd) c_hi = c_hi || br_corner<false>(ring_mask(p, ctr, prm.eps_hi, true), prm.p_min, prm.p_max);
        }
        if (!c_hi && !c_lo) return;
        int score = 0;
#pragma unroll
        for (int j = 0; j < 16; j++) score += abs(p[j] - ctr);
        if (crf && c_hi) crf[lv.crf_offset + (int64_t)(y0 + r) * lv.w + (x0 + col)] = (uint16_t)score;
        const int kx = col / c, ky = r / c;
        const int k = ky * it.nkx + kx;
        if (s_run[k]) {
            const uint32_t off = (uint32_t)((r - ky * c) * c + (col - kx * c));
            const uint32_t key = ((uint32_t)score << 10) | (1023u - off);
            if (c_hi) atomicMax(&s_hi[k], key);
            if (c_lo) atomicMax(&s_lo[k], key);
        }
    };

    // 3b. screen every candidate densely: a run >= p_min at the weaker
    //     threshold is necessary for a corner at either threshold.  Survivors
    //     (entry = rd << 13 | rb << 12 | row << 7 | column) go to a second queue.
    const int n0 = s_qcnt[0], n1 = n0 + s_qcnt[1], n2 = n1 + s_qcnt[2], total = n2 + s_qcnt[3];
    for (int i = tid; i < total; i += 256) {
        const int w = (i >= n0) + (i >= n1) + (i >= n2);
        const int base = w == 0 ? 0 : (w == 1 ? n0 : (w == 2 ? n1 : n2));
        const int e = s_q[w * FT_QSEG + (i - base)];
        const int r = (e >> 7) & 63, col = e & 127;
        const bool pb = (e >> 13) & 1, pd = (e >> 14) & 1;
        int p[16];
        const int ctr = load_ring(r, col, p);
        bool rb = false, rd = false;
        if constexpr (P9) {
            rb = pb && run_ge<true>(ring_mask(p, ctr, prm.eps_min, false), 9);
            // both polarities passed the compass test (rare): try dark only if bright failed
            const bool try_d = pd && !rb;
            if (try_d) rd = run_ge<true>(ring_mask(p, ctr, prm.eps_min, true), 9);
        } else {
            if (pb) rb = run_ge<false>(ring_mask(p, ctr, prm.eps_min, false), prm.p_min);
            if (pd) rd = run_ge<false>(ring_mask(p, ctr, prm.eps_min, true), prm.p_min);
        }
        const bool surv = rb || rd;
        const uint64_t bal = __ballot(surv);
        if (bal) {
            int wbase = 0;
            if (lane == __builtin_ffsll((long long)bal) - 1) wbase = atomicAdd(&s_n2, __popcll(bal));
            wbase = __shfl(wbase, __builtin_ffsll((long long)bal) - 1);
            const int pos = wbase + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
            if (surv) {
                if (pos < FT_Q2) s_q2[pos] = (uint16_t)((rd ? 1 << 13 : 0) | (rb ? 1 << 12 : 0) | (r << 7) | col);
                else finish(r, col, rb, rd);       // queue full: decide in place
            }
        }
    }
    __syncthreads();
    // 3c. decide the survivors densely
    const int ns = min(s_n2, FT_Q2);
    for (int i = tid; i < ns; i += 256) {
        const int e = s_q2[i];
        finish((e >> 7) & 31, e & 127, (e >> 12) & 1, (e >> 13) & 1);
    }
    __syncthreads();
    for (int k = tid; k < nk; k += 256) {
        const uint32_t hi = s_hi[k], lo = s_lo[k];
        const uint32_t v = hi ? hi : (lo ? (lo | VSFE_KEY_FALLBACK) : 0u);
        cell_keys[lv.cell_offset + (int64_t)(it.cy0 + k / it.nkx) * lv.ncx + (it.cx0 + k % it.nkx)] = v;
    }
}

// Zero fill of the optional response dump (no hipMemset, graph friendly).
__global__ void fill_u16_kernel(uint16_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int PF, bool LO>
static void launch_fast(const vsfe_batch *b, hipStream_t st, const uint8_t *images, const uint8_t *pyr,
                        const uint8_t *mask, uint32_t *keys, uint16_t *crf, const DetParams &prm) {
    if (prm.p_min == 9 && prm.p_max == 13)
        hipLaunchKernelGGL((fast_br_kernel<PF, LO, true>), dim3(b->n_det_items), dim3(256), 0, st, b->d_images,
                           b->d_det_items, images, pyr, mask, keys, crf, prm);
    else
        hipLaunchKernelGGL((fast_br_kernel<PF, LO, false>), dim3(b->n_det_items), dim3(256), 0, st, b->d_images,
                           b->d_det_items, images, pyr, mask, keys, crf, prm);
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t fast_br_detect(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                  const uint8_t *pyr, const uint8_t *cell_mask, uint32_t *cell_keys,
                                  uint16_t *crf_debug, int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !cell_keys || (!pyr && b->info.n_levels > 1)) return fail(VSFE_EINVAL, "null buffer");
    const vsfe_params &p = ctx->p;
    DetParams prm;
    prm.eps_hi = p.eps_hi;
    prm.eps_lo = p.eps_lo;
    prm.p_min = p.p_min;
    prm.p_max = p.p_max;
    prm.border = p.border;
    prm.eps_min = p.eps_lo >= 0 ? p.eps_lo : p.eps_hi;
    prm.aligned = b->aligned_input16 && (((uintptr_t)images & 15) == 0) ? 1 : 0;
    const int pf = p.p_min >= 9 ? 2 : (p.p_min >= 5 ? 1 : 0);
    const bool lo = p.eps_lo >= 0;
    hipStream_t st = (hipStream_t)stream;
    if (crf_debug && b->info.crf_elems > 0) {
        hipLaunchKernelGGL(fill_u16_kernel, dim3(1024), dim3(256), 0, st, crf_debug, (int64_t)b->info.crf_elems);
        rc = check_launch("fast_br_detect (response dump fill)");
        if (rc) return rc;
    }
    if (b->n_det_items <= 0) return VSFE_OK;
    if (pf == 2 && lo) launch_fast<2, true>(b, st, images, pyr, cell_mask, cell_keys, crf_debug, prm);
    else if (pf == 2) launch_fast<2, false>(b, st, images, pyr, cell_mask, cell_keys, crf_debug, prm);
    else if (pf == 1 && lo) launch_fast<1, true>(b, st, images, pyr, cell_mask, cell_keys, crf_debug, prm);
    else if (pf == 1) launch_fast<1, false>(b, st, images, pyr, cell_mask, cell_keys, crf_debug, prm);
    else if (lo) launch_fast<0, true>(b, st, images, pyr, cell_mask, cell_keys, crf_debug, prm);
    else launch_fast<0, false>(b, st, images, pyr, cell_mask, cell_keys, crf_debug, prm);
    return check_launch("fast_br_detect");
}
