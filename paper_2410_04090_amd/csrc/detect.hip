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
//     are fetched as 16-byte chunks (one per half per thread, all in flight
//     together) and split with v_perm; the run flags of the learned gate
//     are loaded with them.
//  2. Prefilter every pixel pair with packed 16-bit min / max / saturating
//     subtract: a cyclic run of >= 9 ring pixels covers two adjacent compass
//     pixels (0, 4, 8, 12), i.e. one of {0, 8} and one of {4, 12}, so a
//     bright run needs min(max(p0, p8), max(p4, p12)) > c + eps (dark:
//     max(min(p0, p8), min(p4, p12)) < c - eps), at the weaker threshold.
//  3. Each lane collects its candidates in a bit mask over its rows; a wave
//     prefix sum of the counts on the DPP network places them in the wave's
//     own LDS queue, so the full ring test runs densely over candidates only
//     and no block barrier is needed until the cell keys are reduced.  The
//     screen (a run >= p_min at the weaker threshold, polarity re-derived
//     from the same compass test) compacts its survivors in place; the
//     decision at both thresholds and the response run on the survivors.
//     Ring masks are built with alignbit (one op inserts one sign bit; run
//     lengths do not depend on bit order) and runs are tested by shift-and
//     doubling.
//  4. Keys reduce per cell with LDS atomicMax (order independent, so the
//     result is exact and deterministic) and are written once per cell.
#include "vsfe_internal.h"

namespace vsfe {

constexpr int FT_HALF = 64;                      // lanes per row; lane owns cols l and l + 64
constexpr int FT_CHUNKS = 6;                     // 16-byte source chunks per row and half
// LDS words per row: the 6 staged 16-byte chunks of each half (96 words),
// padded to 100 so that successive rows start 4 banks apart (fewer bank
// conflicts when a wave's candidates sit in the same columns of different rows)
constexpr int FT_W = 100;
constexpr int FT_MAX_ROWS = DET_MAX_TILE_H;
constexpr int FT_ROWS = FT_MAX_ROWS + 6;
constexpr int FT_MAX_CELLS = 32 * DET_MAX_CELLS_Y; // at most 32 x DET_WAVES cells per tile
constexpr int FT_QW = 384;                                // one wave's candidate queue (more: in rounds)
constexpr int FT_DQ = 128;                                // one wave's deferred second-polarity list

struct DetParams {
    int eps_hi, eps_lo, p_min, p_max, border, eps_min, aligned;
};

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ us2 as_us2(uint32_t v) { return __builtin_bit_cast(us2, v); }
__device__ __forceinline__ uint32_t as_u32(us2 v) { return __builtin_bit_cast(uint32_t, v); }

// ring offsets (dx, dy) in cyclic order (compile-time, so that every ring
// read is one LDS access with an immediate offset)
constexpr int kRingDx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
constexpr int kRingDy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

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
    // footprints lie inside the level-0 image, so 32-bit divisions suffice
    const int ic0 = (int)c0;
    int a0 = (int)fx0 / ic0, a1 = (int)(fx1 - 1) / ic0, b0 = (int)fy0 / ic0, b1 = (int)(fy1 - 1) / ic0;
    a1 = a1 < l0.ncx - 1 ? a1 : l0.ncx - 1;
    b1 = b1 < l0.ncy - 1 ? b1 : l0.ncy - 1;
    for (int y = b0; y <= b1; y++)
        for (int x = a0; x <= a1; x++)
            if (mask0[y * l0.ncx + x]) return true;
    return false;
}

// Expand the level-0 cell mask to run flags of every cell of every level
// (one thread per cell), so the detector reads one byte per cell; a cell
// that does not run gets its (empty) key here, since the detector visits
// only tiles with a running cell.  Block 0 also clears the work list's count.
__global__ __launch_bounds__(256) void expand_mask_kernel(const ImageDev *__restrict__ imgs,
                                                          const CellChunk *__restrict__ chunks,
                                                          const uint8_t *__restrict__ mask0,
                                                          uint8_t *__restrict__ run, uint32_t *__restrict__ keys,
                                                          int32_t *__restrict__ list, int level_begin, int level_end) {
    if (blockIdx.x == 0 && threadIdx.x == 0) list[0] = 0;
    const CellChunk ch = chunks[blockIdx.x];
    if (ch.level < level_begin || ch.level >= level_end) return;
    const ImageDev &im = imgs[ch.image];
    const LevelDev lv = im.lv[ch.level];
    const int idx = (int)ch.first + (int)threadIdx.x;
    if (idx >= lv.ncx * lv.ncy) return;
    const int cy = idx / lv.ncx, cx = idx - cy * lv.ncx;
    const bool r = cell_runs(mask0 + im.cell0_offset, im.lv[0], lv, cx, cy);
    run[lv.cell_offset + idx] = r ? 1 : 0;
    if (!r) keys[lv.cell_offset + idx] = 0;
}

// Work list of the gated detector: the items (tiles) with at least one
// running cell, as indices into the launched item range.  One thread per
// item; each block appends its items in order at a position taken with one
// atomic add (the order of blocks in the list does not matter: every item
// writes only its own cells).
__global__ __launch_bounds__(256) void gate_items_kernel(const DetItem *__restrict__ items, int n_items,
                                                         const uint8_t *__restrict__ run, int32_t *__restrict__ list) {
    __shared__ int s_wave[4];
    __shared__ int s_base;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bool any = false;
    if (i < n_items) {
        const DetItem it = items[i];
        for (int ky = 0; ky < it.nky && !any; ky++) {
            const uint8_t *row = run + it.cell_offset + (int64_t)(it.cy0 + ky) * it.ncx + it.cx0;
            for (int kx = 0; kx < it.nkx; kx++) any = any || row[kx] != 0;
        }
    }
    const uint64_t bal = __ballot(any);
    const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
    if (lane == 0) s_wave[wave] = __popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int tot = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
        s_base = tot ? atomicAdd(&list[0], tot) : 0;
    }
    __syncthreads();
    int before = s_base;
    for (int w = 0; w < wave; w++) before += s_wave[w];
    if (any) list[1 + before + below] = i;
}

// 16 consecutive bytes of a row starting at x (zero outside [0, w)).  In
// aligned mode x is a multiple of 16 and the row pitch a multiple of 16 that
// is >= w, so a chunk that starts inside the row is one aligned 16-byte load
// (bytes past w are masked); otherwise bytes are read one by one.
__device__ __forceinline__ uint4 fetch16(const uint8_t *row, int x, int w, bool aligned) {
    if (aligned) {
        if (x < 0 || x >= w) return make_uint4(0, 0, 0, 0);
        uint4 v = *(const uint4 *)(row + x);
        const int valid = w - x;
        if (valid < 16) {
            auto keep = [&](int i) {
                const int k = valid - 4 * i;
                return k >= 4 ? 0xFFFFFFFFu : (k <= 0 ? 0u : (1u << (8 * k)) - 1u);
            };
            v.x &= keep(0);
            v.y &= keep(1);
            v.z &= keep(2);
            v.w &= keep(3);
        }
        return v;
    }
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

// Inclusive prefix sum over the 64 lanes of a wave on the DPP network
// (row shifts within 16-lane rows, then row broadcasts), no LDS round trip.
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31 into rows 2, 3
    return v;
}

// LDS writes of this wave are visible to its later LDS reads (a wave's LDS
// operations complete in order; this stops the compiler from moving reads up)
__device__ __forceinline__ void wave_lds_fence() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// ceil(2^16 / d) for d = 1..32 (cell sides and cells per tile row): for
// v < 2048, (v * ceil(2^16 / d)) >> 16 = v / d exactly.
struct InvTable {
    uint32_t v[33];
};
constexpr InvTable make_inv_table() {
    InvTable t{};
    for (uint32_t d = 1; d <= 32; d++) t.v[d] = (65535u + d) / d;
    return t;
}
__constant__ InvTable c_inv16 = make_inv_table();

template <int PF, bool LO, bool P9>
__global__ __launch_bounds__(DET_THREADS, 32 / DET_WAVES) void fast_br_kernel(const ImageDev *__restrict__ imgs,
                                                      const DetItem *__restrict__ items,
                                                      const uint8_t *__restrict__ images,
                                                      const uint8_t *__restrict__ pyr,
                                                      const uint8_t *__restrict__ mask,
                                                      uint32_t *__restrict__ cell_keys,
                                                      uint16_t *__restrict__ crf,
                                                      const int32_t *__restrict__ list, DetParams prm) {
    __shared__ __attribute__((aligned(16))) uint32_t tile[FT_ROWS * FT_W];
    __shared__ uint16_t s_q[DET_WAVES][FT_QW];
    __shared__ uint16_t s_d[DET_WAVES][FT_DQ];
    __shared__ uint32_t s_hi[FT_MAX_CELLS], s_lo[FT_MAX_CELLS];
    __shared__ uint8_t s_run[FT_MAX_CELLS];
    __shared__ int s_anyw[DET_WAVES];

    // level-major items in dispatch order, in groups of 16 neighbouring
    // tiles per XCD (shared halo lines hit in that XCD's L2; a contiguous
    // range per XCD would give some XCDs only the heavy level 0)
    // (gated: the grid covers every item, the list holds the running ones)
    int item;
    if (list) {
        const int n_run = list[0];
        if ((int)blockIdx.x >= n_run) return;
        item = list[1 + xcd_group_item<16>(blockIdx.x, n_run)];
    } else {
        item = xcd_group_item<16>(blockIdx.x, gridDim.x);
    }
    const DetItem it = items[item];
    const DetItem &lv = it;                      // the level's geometry travels with the item
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int c = lv.cell;
    const int nk = it.nkx * it.nky;
    const uint32_t inv_c = c_inv16.v[c], inv_nkx = c_inv16.v[it.nkx];   // c, nkx <= 32
    // global index of cell k of the tile (k < 2048, so k / nkx is exact by the reciprocal)
    auto cell_index = [&](int k) {
        const int ky = (int)(__umul24((uint32_t)k, inv_nkx) >> 16), kx = k - ky * it.nkx;
        return lv.cell_offset + (int64_t)(it.cy0 + ky) * lv.ncx + (it.cx0 + kx);
    };
    const int x0 = it.cx0 * c, y0 = it.cy0 * c;
    const int x1 = min(x0 + it.nkx * c, lv.w), y1 = min(y0 + it.nky * c, lv.h);
    const int tw = x1 - x0, th = y1 - y0;

    // 1. stage rows y0-3 .. y1+2; word column j holds image columns xb + j and
    //    xb + 64 + j.  One task = one 16-byte chunk of both halves of a row, so
    //    every thread has its two loads in flight at once.  Cell state is
    //    cleared meanwhile (learned gating: which cells run at all).
    const uint8_t *src = (it.level == 0 ? images : pyr) + lv.offset;
    const int xb = (x0 - 3) & ~15, delta = (x0 - 3) - xb;
    const bool aligned = it.level > 0 || prm.aligned != 0;
    // run flags of cells tid and tid + 256, loaded together with the rows
    // (one memory round trip)
    uint32_t mf0 = 1u, mf1 = 1u;
    if (mask) {
        const int k0 = tid, k1 = tid + DET_THREADS;
        mf0 = k0 < nk ? mask[cell_index(k0)] : 0u;
        mf1 = k1 < nk ? mask[cell_index(k1)] : 0u;
    }
    // an interior tile (every staged chunk inside the level, aligned rows)
    // loads without per-thread checks (uniform)
    const bool interior = aligned && xb >= 0 && xb + FT_HALF + 16 * FT_CHUNKS <= lv.w && y0 >= 3 &&
                          y0 + th + 3 <= lv.h;
    if (tid < (th + 6) * FT_CHUNKS) {
        const int rr = tid / FT_CHUNKS, m = tid - rr * FT_CHUNKS;
        const int gy = y0 - 3 + rr;
        uint4 L, R;
        if (interior) {
            const uint8_t *row = src + (int64_t)gy * lv.pitch + xb + 16 * m;
            L = *(const uint4 *)row;
            R = *(const uint4 *)(row + FT_HALF);
        } else {
            L = make_uint4(0, 0, 0, 0);
            R = make_uint4(0, 0, 0, 0);
            if (gy >= 0 && gy < lv.h) {
                const uint8_t *row = src + (int64_t)gy * lv.pitch;
                L = fetch16(row, xb + 16 * m, lv.w, aligned);
                R = fetch16(row, xb + FT_HALF + 16 * m, lv.w, aligned);
            }
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
    int my_any = 0;
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int k = tid + DET_THREADS * h;
        if (k < nk) {
            const bool run = (h ? mf1 : mf0) != 0u;
            s_run[k] = run;
            s_hi[k] = 0;
            s_lo[k] = 0;
            my_any |= run;
        }
    }
    if (mask) {
        // does any cell of the tile run: one flag per wave, one barrier
        const bool wave_any = __ballot(my_any) != 0;
        if (lane == 0) s_anyw[wave] = wave_any;
        __syncthreads();
        int any = 0;
#pragma unroll
        for (int w = 0; w < DET_WAVES; w++) any |= s_anyw[w];
        if (!any && !crf) {
            for (int k = tid; k < nk; k += DET_THREADS)
                cell_keys[cell_index(k)] = 0;
            return;
        }
    } else {
        __syncthreads();
    }

    // From here until the cell keys are reduced every wave works alone on
    // its rows (wave + 4k): its own candidate and survivor queues, no block
    // barrier.
    //
    // 2. prefilter: each lane collects its candidates in a bit mask: bit k =
    //    column lane of row wave + 4k, bit 16 + k = column lane + 64.
    const int B = prm.border;
    const int gxl = x0 + lane, gxh = x0 + FT_HALF + lane;
    const bool okl = lane < tw && gxl >= B && gxl < lv.w - B;
    const bool okh = FT_HALF + lane < tw && gxh >= B && gxh < lv.w - B;
    const us2 e2 = {(unsigned short)prm.eps_min, (unsigned short)prm.eps_min};
    const int ylo = max(B - y0, 0), yhi = min(lv.h - B - y0, th);
    // v < 2048: (v * ceil(2^16 / d)) >> 16 is v / d exactly (for d <= 32)
    auto div_c = [&](int v) { return (int)(__umul24((uint32_t)v, inv_c) >> 16); };
    const int kxl = div_c(lane), kxh = div_c(FT_HALF + lane);
    uint32_t cm = 0;
    // one base address for all rows of the wave: each row then reads at
    // constant offsets
    const uint32_t *const t0 = &tile[(wv + 3) * FT_W + lane + 3 + delta];
    // the west and east neighbours through base registers of their own: the
    // compiler would otherwise pair one of them with the centre into a
    // ds_read2, whose short offset field costs an address add per row
    int w0 = (wv + 3) * FT_W + lane + delta, e0 = w0 + 6;
    asm volatile("" : "+v"(w0), "+v"(e0));
    // the flag clamp's (1, 1) in a scalar register set once (as a constant
    // the compiler would write it again for every row)
    uint32_t one2;
    asm volatile("s_mov_b32 %0, 0x10001" : "=s"(one2));
    // this wave's rows wv + 4k inside [ylo, yhi): k in [k_lo, k_hi)
    const int k_lo = max(ylo - wv + DET_WAVES - 1, 0) / DET_WAVES;
    const uint32_t k_n = (uint32_t)max((yhi - wv + DET_WAVES - 1) / DET_WAVES - k_lo, 0);
#pragma unroll
    for (int k = 0; k < FT_MAX_ROWS / DET_WAVES; k++) {
        if ((uint32_t)(k - k_lo) >= k_n) continue;                    // uniform
        const uint32_t *t = t0 + DET_WAVES * FT_W * k;
        uint32_t f = 0x10001u;                    // (low, high) candidate flags
        if (PF) {
            const us2 C = as_us2(t[0]);
            const us2 P0 = as_us2(t[-3 * FT_W]), P8 = as_us2(t[3 * FT_W]);
            const us2 P4 = as_us2(tile[e0 + DET_WAVES * FT_W * k]), P12 = as_us2(tile[w0 + DET_WAVES * FT_W * k]);
            us2 Mb, Md;
            if (PF == 2) {
                Mb = __builtin_elementwise_min(__builtin_elementwise_max(P0, P8), __builtin_elementwise_max(P4, P12));
                Md = __builtin_elementwise_max(__builtin_elementwise_min(P0, P8), __builtin_elementwise_min(P4, P12));
            } else {
                Mb = __builtin_elementwise_max(__builtin_elementwise_max(P0, P8), __builtin_elementwise_max(P4, P12));
                Md = __builtin_elementwise_min(__builtin_elementwise_min(P0, P8), __builtin_elementwise_min(P4, P12));
            }
            // Mb > C + eps or Md < C - eps, i.e. max(Mb - C, C - Md) > eps
            // with both differences clamped at zero
            const us2 d = __builtin_elementwise_max(__builtin_elementwise_sub_sat(Mb, C),
                                                    __builtin_elementwise_sub_sat(C, Md));
            // (low != 0, high != 0) of d - eps as two 16-bit flags in one
            // v_pk_min_u16 (in asm: the compiler would otherwise expand it
            // into compares and selects)
            const uint32_t x = as_u32(__builtin_elementwise_sub_sat(d, e2));
            asm volatile("v_pk_min_u16 %0, %1, %2" : "=v"(f) : "v"(x), "s"(one2));
        }
        cm |= f << k;
    }
    cm &= (okl ? 0xFFu : 0u) | (okh ? 0xFF0000u : 0u);
    if (mask) {
        // learned gating: pixels of skipped cells never become candidates
        const int ka = min(kxl, it.nkx - 1), kb = min(kxh, it.nkx - 1);
        uint32_t gm = 0;
        if (it.nky == 1) {                               // one cell row (levels with c >= 16): per lane
            gm = (s_run[ka] ? 0xFFu : 0u) | (s_run[kb] ? 0xFF0000u : 0u);
        } else {
            // run flags of the lane's two cells in each cell row j (bits j and
            // 8 + j), read once; a pixel row then selects its cell row's bits
            uint32_t rb = 0;
#pragma unroll
            for (int j = 0; j < DET_MAX_CELLS_Y; j++) {
                if (j >= it.nky) break;                  // uniform
                rb |= (s_run[j * it.nkx + ka] ? 1u : 0u) << j;
                rb |= (s_run[j * it.nkx + kb] ? 0x100u : 0u) << j;
            }
#pragma unroll
            for (int k = 0; k < FT_MAX_ROWS / DET_WAVES; k++) {
                const int r = wv + DET_WAVES * k;
                if (r >= th) break;                      // uniform
                const int j = (int)((uint32_t)(r * inv_c) >> 16);              // r < 32: r / c exactly
                gm |= ((rb >> j) & 1u) << k;
                gm |= ((rb >> (8 + j)) & 1u) << (16 + k);
            }
        }
        cm &= gm;
    }

    // 3a. this wave's candidate queue (entry = row << 7 | column): a DPP scan
    //     of the per-lane counts places every lane's entries
    const int cnt = __popc(cm);
    const int incl = wave_incl_scan(cnt);
    const int qn = __builtin_amdgcn_readlane(incl, 63);
    uint16_t *const q = s_q[wv];

    const uint16_t *t16 = (const uint16_t *)tile;
    // the 16 ring pixels and the centre of tile pixel (r, col), from LDS
    auto load_ring = [&](int r, int col, int *p) {
        const uint16_t *win = t16 + 2 * (r * FT_W + (col & 63) + delta) + (col >> 6);
#pragma unroll
        for (int j = 0; j < 16; j++) p[j] = win[2 * ((kRingDy[j] + 3) * FT_W + kRingDx[j] + 3)];
        return (int)win[2 * (3 * FT_W + 3)];
    };
    // decision for a screened pixel: rb / rd = polarities with a run >= p_min at eps_min
    // with p_min = 9 the screen, which runs at eps_min (eps_lo if there is a
    // fallback threshold, else eps_hi), has already taken the corner decision
    // at that threshold (cmin)
    auto decide = [&](const int *p, int ctr, int r, int col, bool rb, bool rd, bool cmin) {
        bool c_hi = false, c_lo = false;
        if constexpr (P9) {
            // p_min = 9: a bright and a dark run cannot coexist, one polarity decides
            if (LO) {
                c_lo = cmin;
                c_hi = br_corner<true>(ring_mask(p, ctr, prm.eps_hi, !rb), 9, 13);
            } else {
                c_hi = cmin;
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
        // response: sum of |I_p - I_c| over the ring, two pixels per v_sad_u16
        const uint32_t c2 = (uint32_t)ctr * 0x10001u;
        uint32_t score = 0;
#pragma unroll
        for (int j = 0; j < 16; j += 2)
            score = __builtin_amdgcn_sad_u16((uint32_t)p[j] | ((uint32_t)p[j + 1] << 16), c2, score);
        if (crf && c_hi) crf[lv.crf_offset + (int64_t)(y0 + r) * lv.w + (x0 + col)] = (uint16_t)score;
        const int kx = div_c(col), ky = div_c(r);                     // col < 128, r < 32
        const int k = ky * it.nkx + kx;
        if (s_run[k]) {
            const uint32_t off = (uint32_t)((r - ky * c) * c + (col - kx * c));
            const uint32_t key = ((uint32_t)score << 10) | (1023u - off);
            if (c_hi) atomicMax(&s_hi[k], key);
            if (c_lo) atomicMax(&s_lo[k], key);
        }
    };
    auto finish = [&](int r, int col, bool rb, bool rd, bool cmin) {
        int p[16];
        const int ctr = load_ring(r, col, p);
        decide(p, ctr, r, col, rb, rd, cmin);
    };

    // The queue holds FT_QW entries; a wave with more candidates (dense
    // texture) takes them in rounds, each screened and decided in full.
    for (int r0 = 0; r0 < qn; r0 += FT_QW) {
    {
        // entry of bit b = 16 h + k: (wv + W k) << 7 | (lane + 64 h)
        //     = base + 128 W k + 4 (b - k) = base + 4 b + (128 W - 4) k
        static_assert(FT_HALF == 64, "entry arithmetic assumes 64-lane halves");
        constexpr int EK = 128 * DET_WAVES - 4;
        const int ebase = (wv << 7) | lane;
        uint32_t mm = cm;
        int pos = incl - cnt;
        if (qn <= FT_QW) {                       // uniform: one round, every entry fits
            while (mm) {
                const int bit = __builtin_ctz(mm);
                mm &= mm - 1;
                q[pos++] = (uint16_t)(ebase + 4 * bit + EK * (bit & 15));
            }
        } else {
            while (mm) {
                const int bit = __builtin_ctz(mm);
                mm &= mm - 1;
                if (pos >= r0 && pos < r0 + FT_QW) q[pos - r0] = (uint16_t)(ebase + 4 * bit + EK * (bit & 15));
                pos++;
            }
        }
    }
    wave_lds_fence();
    const int qr = min(FT_QW, qn - r0);
    // 3b. screen every candidate densely: a run >= p_min at the weaker
    //     threshold is necessary for a corner at either threshold.  Survivors
    //     (entry = cmin << 15 | rd << 14 | rb << 13 | row << 7 | column) go to
    //     a second queue.
    // survivors are compacted in place: after the iteration that reads
    // entries [base, base + 64), at most base + 64 survivors exist, so a
    // survivor never overwrites an entry that is still to be read
    uint16_t *const q2 = q;
    int n2 = 0;                                  // survivors so far (uniform)
    auto emit = [&](bool surv, int entry) {
        const uint64_t bal = __ballot(surv);
        const int pos2 = n2 + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
        if (surv) q2[pos2] = (uint16_t)entry;
        n2 += __popcll(bal);
    };
    // p_min = 9: a lane tests one polarity (bright if it passed the compass
    // test, else dark).  A pixel that passed both and has no bright run (a
    // sixth to a quarter of the candidates, so nearly every batch has one)
    // is deferred to this wave's list and tested dark in dense batches of
    // 64; a deferred pixel's survivor is still at most one output per
    // candidate, so the in-place compaction above stays valid.
    uint16_t *const dq = s_d[wv];
    int nd = 0;                                  // deferred entries (uniform)
    auto screen_dark = [&](int first, int count) {
        const bool a = lane < count;
        const int e = a ? dq[first + lane] : 0;
        int p[16];
        const int ctr = load_ring((e >> 7) & 63, e & 127, p);
        const uint32_t m = ring_mask(p, ctr, prm.eps_min, true);
        const bool run = run_ge<true>(m, 9);
        const bool cmin = run && !run_ge<false>(m, 14);
        emit(a && run, (cmin ? 1 << 15 : 0) | (1 << 14) | (e & 0x1FFF));
    };
    for (int base = 0; base < qr; base += 64) {
        const int i = base + lane;
        const bool act = i < qr;
        const int e = act ? q[i] : 0;
        const int r = (e >> 7) & 63, col = e & 127;
        int p[16];
        const int ctr = load_ring(r, col, p);
        // polarities that passed the prefilter (the same compass test)
        bool pb = true, pd = true;
        if (PF == 2) {
            pb = min(max(p[0], p[8]), max(p[4], p[12])) > ctr + prm.eps_min;
            pd = max(min(p[0], p[8]), min(p[4], p[12])) < ctr - prm.eps_min;
        } else if (PF == 1) {
            pb = max(max(p[0], p[8]), max(p[4], p[12])) > ctr + prm.eps_min;
            pd = min(min(p[0], p[8]), min(p[4], p[12])) < ctr - prm.eps_min;
        }
        bool rb = false, rd = false, cmin = false, defer = false;
        if constexpr (P9) {
            const bool dk = !pb;
            const uint32_t m = ring_mask(p, ctr, prm.eps_min, dk);
            const bool run = run_ge<true>(m, 9);
            defer = act && !run && pb && pd;
            rb = run && !dk;
            rd = run && dk;
            cmin = run && !run_ge<false>(m, 14);
        } else {
            if (pb) rb = run_ge<false>(ring_mask(p, ctr, prm.eps_min, false), prm.p_min);
            if (pd) rd = run_ge<false>(ring_mask(p, ctr, prm.eps_min, true), prm.p_min);
        }
        emit(act && (rb || rd), (cmin ? 1 << 15 : 0) | (rd ? 1 << 14 : 0) | (rb ? 1 << 13 : 0) | (r << 7) | col);
        if constexpr (P9) {
            const uint64_t bd = __ballot(defer);
            if (bd) {                                // uniform
                const int posd = nd + __builtin_amdgcn_mbcnt_hi((uint32_t)(bd >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bd, 0));
                if (defer) dq[posd] = (uint16_t)(e & 0x1FFF);
                nd += __popcll(bd);                  // < 64 before, <= 127 after
                if (nd >= 64) {
                    nd -= 64;
                    wave_lds_fence();
                    screen_dark(nd, 64);
                }
            }
        }
    }
    if (P9 && nd > 0) {
        wave_lds_fence();
        screen_dark(0, nd);
    }
    wave_lds_fence();
    // 3c. decide this wave's survivors densely, then reduce over the block
    const int ns = n2;
    for (int i = lane; i < ns; i += 64) {
        const int e = q2[i];
        finish((e >> 7) & 63, e & 127, (e >> 13) & 1, (e >> 14) & 1, (e >> 15) & 1);
    }
    wave_lds_fence();
    }  // rounds
    __syncthreads();
    for (int k = tid; k < nk; k += DET_THREADS) {       // nk <= 128
        const uint32_t hi = s_hi[k], lo = s_lo[k];
        const uint32_t v = hi ? hi : (lo ? (lo | VSFE_KEY_FALLBACK) : 0u);
        cell_keys[cell_index(k)] = v;
    }
}

// Zero fill of the optional response dump (no hipMemset, graph friendly).
__global__ void fill_u16_kernel(uint16_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

template <int PF, bool LO>
static void launch_fast(const vsfe_batch *b, const DetItem *items, int32_t n_items, hipStream_t st,
                        const uint8_t *images, const uint8_t *pyr, const uint8_t *mask, uint32_t *keys,
                        uint16_t *crf, const int32_t *list, const DetParams &prm) {
    if (prm.p_min == 9 && prm.p_max == 13)
        hipLaunchKernelGGL((fast_br_kernel<PF, LO, true>), dim3(n_items), dim3(DET_THREADS), 0, st, b->d_images, items,
                           images, pyr, mask, keys, crf, list, prm);
    else
        hipLaunchKernelGGL((fast_br_kernel<PF, LO, false>), dim3(n_items), dim3(DET_THREADS), 0, st, b->d_images, items,
                           images, pyr, mask, keys, crf, list, prm);
}

int32_t detect_launch(const vsfe_ctx *ctx, const vsfe_batch *b, const DetItem *items, int32_t n_items,
                      const uint8_t *images, const uint8_t *pyr, const uint8_t *cell_mask, uint32_t *cell_keys,
                      uint16_t *crf_debug, const int32_t *item_list, hipStream_t st) {
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
    if (n_items <= 0) return VSFE_OK;
    if (pf == 2 && lo) launch_fast<2, true>(b, items, n_items, st, images, pyr, cell_mask, cell_keys, crf_debug, item_list, prm);
    else if (pf == 2) launch_fast<2, false>(b, items, n_items, st, images, pyr, cell_mask, cell_keys, crf_debug, item_list, prm);
    else if (pf == 1 && lo) launch_fast<1, true>(b, items, n_items, st, images, pyr, cell_mask, cell_keys, crf_debug, item_list, prm);
    else if (pf == 1) launch_fast<1, false>(b, items, n_items, st, images, pyr, cell_mask, cell_keys, crf_debug, item_list, prm);
    else if (lo) launch_fast<0, true>(b, items, n_items, st, images, pyr, cell_mask, cell_keys, crf_debug, item_list, prm);
    else launch_fast<0, false>(b, items, n_items, st, images, pyr, cell_mask, cell_keys, crf_debug, item_list, prm);
    return check_launch("fast_br_detect");
}

// Gate expansion (if a mask is given) and the detector over the items of
// levels [lb, le).
static int32_t detect_range(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images, const uint8_t *pyr,
                            const uint8_t *cell_mask, uint32_t *cell_keys, uint16_t *crf_debug, int lb, int le,
                            hipStream_t st) {
    const uint8_t *run = nullptr;
    const int32_t *list = nullptr;
    const int i0 = b->det_start[lb], i1 = b->det_start[le];
    if (cell_mask) {
        if (!b->d_run || !b->d_item_list || b->item_list_cap < b->n_det_items)
            return fail(VSFE_EINVAL, "batch has no gating tables");
        if (b->n_chunks > 0) {
            hipLaunchKernelGGL(expand_mask_kernel, dim3(b->n_chunks), dim3(PYCA_CHUNK), 0, st, b->d_images,
                               b->d_chunks, cell_mask, b->d_run, cell_keys, b->d_item_list, lb, le);
            int32_t rc = check_launch("fast_br_detect (mask expansion)");
            if (rc) return rc;
            if (i1 > i0) {
                hipLaunchKernelGGL(gate_items_kernel, dim3((unsigned)((i1 - i0 + 255) / 256)), dim3(256), 0, st,
                                   b->d_det_items + i0, i1 - i0, b->d_run, b->d_item_list);
                rc = check_launch("fast_br_detect (work list)");
                if (rc) return rc;
            }
            list = b->d_item_list;
        }
        run = b->d_run;
    }
    return detect_launch(ctx, b, b->d_det_items + i0, i1 - i0, images, pyr, run, cell_keys, crf_debug, list, st);
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t fast_br_detect(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                  const uint8_t *pyr, const uint8_t *cell_mask, uint32_t *cell_keys,
                                  uint16_t *crf_debug, int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !cell_keys || (!pyr && b->info.n_levels > 1)) return fail(VSFE_EINVAL, "null buffer");
    hipStream_t st = (hipStream_t)stream;
    if (crf_debug && b->info.crf_elems > 0) {
        hipLaunchKernelGGL(fill_u16_kernel, dim3(1024), dim3(256), 0, st, crf_debug, (int64_t)b->info.crf_elems);
        rc = check_launch("fast_br_detect (response dump fill)");
        if (rc) return rc;
    }
    return detect_range(ctx, b, images, pyr, cell_mask, cell_keys, crf_debug, 0, b->info.n_levels, st);
}

extern "C" int32_t fast_br_detect_levels(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                         const uint8_t *pyr, const uint8_t *cell_mask, uint32_t *cell_keys,
                                         int32_t level_begin, int32_t level_end, int32_t *status, void *stream) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (level_begin < 0 || level_end > b->info.n_levels || level_begin >= level_end)
        return fail(VSFE_EINVAL, "level range out of range or empty");
    if (!images || !cell_keys || (!pyr && level_end > 1)) return fail(VSFE_EINVAL, "null buffer");
    return detect_range(ctx, b, images, pyr, cell_mask, cell_keys, nullptr, level_begin, level_end,
                        (hipStream_t)stream);
}
