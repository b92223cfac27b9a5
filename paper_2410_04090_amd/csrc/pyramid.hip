// Image pyramid at scale 1.2 (Sec. III-2): level l is resampled from level
// l-1 by bilinear interpolation at half-pixel centres.  Source coordinates
// are floored to Q8, the four 8-bit weights give a Q16 sum rounded half up:
//   ((256-fx)(256-fy) p_aa + fx (256-fy) p_ab + (256-fx) fy p_ba + fx fy p_bb
//    + 32768) >> 16,
// evaluated here as a horizontal then a vertical integer lerp (the same
// exact sum, factored: h = 256 a + fx (b - a), v = 256 h0 + fy (h1 - h0)).
//
// Two schedules build the same bytes.  Per level (large batches, where
// the launches stream HBM): one launch per level covers that level of every
// image.  Single launch (small and mixed batches, where seven dependent
// launches dominate): pyramid_tower_kernel below builds every level of a
// tile in LDS from one level-0 window.
//
// Per-level schedule: a block writes a
// 256 x 32 output tile: it stages the source window (chosen on the host, at
// most 336 x 44 bytes) in LDS with 16-byte loads and reads per-column and
// per-row source indices and weights from host-built tables (no division on
// the device).  Each lane produces 4 columns of its wave's 8 rows, so the
// source rows are uniform per wave: every needed source row is lerped
// horizontally once, two columns per packed 16-bit multiply-add
// (a (256 - fx) + b fx <= 65280 fits), with the 4 source bytes of a column
// pair gathered by one v_perm from two LDS dwords; the vertical lerp is one
// v_dot2_u32_u16 per output (its top / bottom pair gathered by one v_perm)
// whose byte 2 is the rounded result, and the 4 outputs are stored as one
// 32-bit word.
#include "vsfe_internal.h"

namespace vsfe {

constexpr int PYR_LDS_W = PYR_SW + 16;  // padded row stride (bank spread), 16-byte aligned
constexpr int PYR_TASKS = (PYR_SH * (PYR_SW / 16) + 255) / 256;

typedef unsigned short pu2 __attribute__((ext_vector_type(2)));

// Vertical lerp of four columns: byte 2 of h_top (256 - fy) + h_bot fy +
// 2^15 (< 2^24) per column, from the horizontal lerps of the top and bottom
// source rows as u16 pairs (t01, t23 / u01, u23).  Each column's (top,
// bottom) pair is gathered into one register by v_perm and weighted by one
// v_dot2_u32_u16 against wf = (256 - fy, fy); the four bytes 2 pack into a
// word.
__device__ __forceinline__ uint32_t vlerp4(pu2 t01, pu2 t23, pu2 u01, pu2 u23, uint32_t wf) {
    const pu2 W = __builtin_bit_cast(pu2, wf);
    const uint32_t a01 = __builtin_bit_cast(uint32_t, t01), b01 = __builtin_bit_cast(uint32_t, u01);
    const uint32_t a23 = __builtin_bit_cast(uint32_t, t23), b23 = __builtin_bit_cast(uint32_t, u23);
    const uint32_t s0 = __builtin_amdgcn_udot2(__builtin_bit_cast(pu2, __builtin_amdgcn_perm(b01, a01, 0x05040100u)), W, 32768u, false);
    const uint32_t s1 = __builtin_amdgcn_udot2(__builtin_bit_cast(pu2, __builtin_amdgcn_perm(b01, a01, 0x07060302u)), W, 32768u, false);
    const uint32_t s2 = __builtin_amdgcn_udot2(__builtin_bit_cast(pu2, __builtin_amdgcn_perm(b23, a23, 0x05040100u)), W, 32768u, false);
    const uint32_t s3 = __builtin_amdgcn_udot2(__builtin_bit_cast(pu2, __builtin_amdgcn_perm(b23, a23, 0x07060302u)), W, 32768u, false);
    return __builtin_amdgcn_perm(s1, s0, 0x0C0C0602u) | (__builtin_amdgcn_perm(s3, s2, 0x0C0C0602u) << 16);
}

// 16 consecutive bytes of a row from x, coordinates clamped to [0, w).
__device__ __forceinline__ uint4 fetch16c(const uint8_t *row, int x, int w, bool aligned) {
    if (aligned && x >= 0 && x + 15 < w) return *(const uint4 *)(row + x);
    uint32_t v[4] = {0, 0, 0, 0};
    for (int j = 0; j < 16; j++) v[j >> 2] |= (uint32_t)row[min(max(x + j, 0), w - 1)] << (8 * (j & 3));
    return make_uint4(v[0], v[1], v[2], v[3]);
}

__global__ __launch_bounds__(256) void pyramid_level_kernel(const ImageDev *__restrict__ imgs,
                                                            const PyrItem *__restrict__ items, int level,
                                                            const uint32_t *__restrict__ coord,
                                                            const uint8_t *__restrict__ images,
                                                            uint8_t *__restrict__ pyr, int aligned0) {
    __shared__ __attribute__((aligned(16))) uint32_t s_src[PYR_SH * (PYR_LDS_W / 4)];
    const PyrItem it = items[xcd_item(blockIdx.x, gridDim.x)];
    const struct { int w, h, pitch; int64_t offset; } s = {it.sw, it.sh, it.spitch, it.src_offset};
    const struct { int w, h, pitch, xtab, ytab; int64_t offset; } d = {it.dw, it.dh, it.dpitch, it.xtab, it.ytab,
                                                                      it.dst_offset};
    const uint8_t *src = (level == 1 ? images : pyr) + s.offset;
    uint8_t *dst = pyr + d.offset;
    const int tid = threadIdx.x;
    const bool aligned = level > 1 || aligned0;

    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    constexpr int ROWS = PYR_TH / 4;                     // output rows per wave
    const int oy0 = it.ty * PYR_TH + ROWS * wave;        // uniform
    const int ox = it.tx * PYR_TW + 4 * lane;
    // resampling table entries of the lane's 4 columns and the wave's rows,
    // loaded together with the staged rows
    uint32_t ex[4], ey[ROWS];
#pragma unroll
    for (int j = 0; j < 4; j++) ex[j] = coord[d.xtab + min(ox + j, d.w - 1)];
#pragma unroll
    for (int k = 0; k < ROWS; k++) ey[k] = coord[d.ytab + min(oy0 + k, d.h - 1)];

    // stage rows ys .. ys+nrows-1, columns xs .. xs+ncols-1 (clamped to the
    // level) as 16-byte chunks, task q = row q / 21, chunk q % 21 (a
    // constant divisor); all of a thread's loads are issued before any LDS
    // store so they are in flight together
    constexpr int CPR = PYR_SW / 16;
    uint4 v[PYR_TASKS];
    int at[PYR_TASKS];
#pragma unroll
    for (int u = 0; u < PYR_TASKS; u++) {
        const int q = tid + 256 * u;
        const int rr = q / CPR, k = q - rr * CPR;
        at[u] = -1;
        if (rr < it.nrows && 16 * k < it.ncols) {
            const int gy = min(it.ys + rr, s.h - 1);
            v[u] = fetch16c(src + (int64_t)gy * s.pitch, it.xs + 16 * k, s.w, aligned);
            at[u] = rr * (PYR_LDS_W / 16) + k;
        }
    }
#pragma unroll
    for (int u = 0; u < PYR_TASKS; u++)
        if (at[u] >= 0) ((uint4 *)s_src)[at[u]] = v[u];
    __syncthreads();

    if (oy0 >= d.h) return;
    // columns: source index (window-local) and weight of the lane's 4 outputs
    int o[4], fx[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        o[j] = (int)(ex[j] & 0xFFFFu) - it.xs;
        fx[j] = (int)(ex[j] >> 16);
    }
    // byte selectors of (a0, a1), (b0, b1), (a2, a3), (b2, b3) within the
    // two dwords at base01 / base23 (0x0c selects a zero byte)
    const int base01 = o[0] & ~3, base23 = o[2] & ~3;
    const uint32_t selA01 = (uint32_t)(o[0] - base01) | 0x0C00u | ((uint32_t)(o[1] - base01) << 16) | 0x0C000000u;
    const uint32_t selA23 = (uint32_t)(o[2] - base23) | 0x0C00u | ((uint32_t)(o[3] - base23) << 16) | 0x0C000000u;
    const uint32_t selB01 = selA01 + 0x00010001u, selB23 = selA23 + 0x00010001u;
    const pu2 W01 = {(unsigned short)(256 - fx[0]), (unsigned short)(256 - fx[1])};
    const pu2 W23 = {(unsigned short)(256 - fx[2]), (unsigned short)(256 - fx[3])};
    const pu2 F01 = {(unsigned short)fx[0], (unsigned short)fx[1]};
    const pu2 F23 = {(unsigned short)fx[2], (unsigned short)fx[3]};
    const uint8_t *sb = (const uint8_t *)s_src;
    // horizontal lerps (x 256) of window row ya for the 4 columns, as two u16 pairs
    auto hrow = [&](int ya, pu2 &h01, pu2 &h23) {
        const uint8_t *r = sb + ya * PYR_LDS_W;
        const uint32_t d0 = *(const uint32_t *)(r + base01), d1 = *(const uint32_t *)(r + base01 + 4);
        const uint32_t e0 = *(const uint32_t *)(r + base23), e1 = *(const uint32_t *)(r + base23 + 4);
        const pu2 A01 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(d1, d0, selA01));
        const pu2 B01 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(d1, d0, selB01));
        const pu2 A23 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(e1, e0, selA23));
        const pu2 B23 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(e1, e0, selB23));
        h01 = A01 * W01 + B01 * F01;
        h23 = A23 * W23 + B23 * F23;
    };
    // output rows at 32-bit byte offsets from the level's uniform first byte
    // (a level of the pyramid buffer holds fewer than 2^27 bytes)
    typedef __attribute__((address_space(1))) uint8_t gbyte;
    typedef __attribute__((address_space(1))) uint32_t gword;
    gbyte *const obase = (gbyte *)dst;
    uint32_t ooff = __umul24((uint32_t)oy0, (uint32_t)d.pitch) + (uint32_t)ox;
    int cur = -2;
    pu2 t01, t23, u01, u23;                              // rows cur, cur + 1
#pragma unroll
    for (int k = 0; k < ROWS; k++) {
        const int oy = oy0 + k;
        if (oy >= d.h) break;                            // uniform
        const uint32_t e = ey[k];
        const int ya = (int)(e & 0xFFFFu) - it.ys;
        const uint32_t fy = e >> 16, wf = (256u - fy) | (fy << 16);
        if (ya == cur + 1) {                             // slide by one row
            t01 = u01;
            t23 = u23;
            hrow(ya + 1, u01, u23);
        } else if (ya != cur) {
            hrow(ya, t01, t23);
            hrow(ya + 1, u01, u23);
        }
        cur = ya;
        // (h0 (256 - fy) + h1 fy + 2^15) >> 16 is byte 2 of the sum
        const uint32_t word = vlerp4(t01, t23, u01, u23, wf);
        if (ox + 3 < d.w) {
            *(gword *)(obase + ooff) = word;
        } else {
            for (int j = 0; ox + j < d.w; j++) obase[ooff + j] = (uint8_t)(word >> (8 * j));
        }
        ooff += (uint32_t)d.pitch;
    }
}


// Single-launch schedule.  A block stages its level-0 window (16-byte
// chunks), its two plans' resampling tables and the level records in LDS,
// then builds levels 1 .. L-1 in turn from the level above, ping-ponging
// between two LDS buffers (even levels at 0, odd ones at odd_off): every
// computed pixel goes to LDS for the next level, the owned ones also to
// HBM.  A level's quads (4 columns) go to groups of QL lanes (QL = the
// power of two >= quads, at least 8), each group a run of consecutive rows
// so that the horizontal lerp of a source row is reused by the next output
// row, as in the per-level kernel.  Source reads past a range (the right /
// bottom neighbour of the last column / row) only happen with weight 0 and
// stay inside the buffer's padding (4 columns, 1 row; 16 columns at level 0).
__global__ __launch_bounds__(256) void pyramid_tower_kernel(const ImageDev *__restrict__ imgs,
                                                            const TowerItem *__restrict__ items,
                                                            const TowerAxis *__restrict__ axes,
                                                            const uint32_t *__restrict__ ttab, int L, int tab_cap,
                                                            const uint8_t *__restrict__ images,
                                                            uint8_t *__restrict__ pyr, int aligned0) {
    extern __shared__ __attribute__((aligned(16))) uint32_t s_dyn[];
    __shared__ TowerAxis s_ax[2];
    __shared__ int64_t s_off[VSFE_MAX_LEVELS];
    __shared__ int32_t s_pitch[VSFE_MAX_LEVELS], s_w[VSFE_MAX_LEVELS];
    uint32_t *s_tab = s_dyn;
    uint8_t *pool = (uint8_t *)(s_dyn + tab_cap);
    const TowerItem it = items[xcd_item(blockIdx.x, gridDim.x)];
    const int tid = threadIdx.x;

    // every global read of the block is issued before the first LDS store
    const uint8_t *src = images + it.src_offset;
    const int S0 = it.ncols + 16;
    const int cpr = it.ncols >> 4;
    uint4 v[TWR_STAGE];
    int at[TWR_STAGE];
#pragma unroll
    for (int u = 0; u < TWR_STAGE; u++) {
        const int q = tid + 256 * u;
        const int rr = q / cpr, k = q - rr * cpr;
        at[u] = -1;
        if (rr < it.nrows) {
            const int gy = min(it.ys + rr, it.sh - 1);
            v[u] = fetch16c(src + (int64_t)gy * it.spitch, it.xs + 16 * k, it.sw, aligned0 != 0);
            at[u] = rr * (S0 >> 4) + k;
        }
    }
    constexpr int TPT = TWR_TAB / 256;
    const int ntab = it.ntabx + it.ntaby;
    uint32_t tv[TPT];
#pragma unroll
    for (int u = 0; u < TPT; u++) {
        const int e = tid + 256 * u;
        tv[u] = 0;
        if (e < ntab) tv[u] = ttab[e < it.ntabx ? it.tabx + e : it.taby + (e - it.ntabx)];
    }
    constexpr int AXW = (int)sizeof(TowerAxis) / 4;
    uint32_t axv = 0;
    if (tid < 2 * AXW) axv = ((const uint32_t *)(axes + (tid < AXW ? it.ax : it.ay)))[tid % AXW];
    int64_t lo = 0;
    int32_t lp = 0, lw = 0;
    if (tid < L) {
        const LevelDev &lv = imgs[it.image].lv[tid];
        lo = lv.offset;
        lp = lv.pitch;
        lw = lv.w;
    }
#pragma unroll
    for (int u = 0; u < TWR_STAGE; u++)
        if (at[u] >= 0) ((uint4 *)pool)[at[u]] = v[u];
#pragma unroll
    for (int u = 0; u < TPT; u++)
        if (tid + 256 * u < ntab) s_tab[tid + 256 * u] = tv[u];
    if (tid < 2 * AXW) ((uint32_t *)s_ax)[tid] = axv;
    if (tid < L) {
        s_off[tid] = lo;
        s_pitch[tid] = lp;
        s_w[tid] = lw;
    }

    int xoff = 0, yoff = it.ntabx;
    int src_stride = S0;
    for (int l = 1; l < L; l++) {
        __syncthreads();
        const int cw = __builtin_amdgcn_readfirstlane(s_ax[0].cn[l]);
        const int ch = __builtin_amdgcn_readfirstlane(s_ax[1].cn[l]);
        const int cx0 = __builtin_amdgcn_readfirstlane(s_ax[0].c0[l]);
        const int cy0 = __builtin_amdgcn_readfirstlane(s_ax[1].c0[l]);
        const int ox0 = __builtin_amdgcn_readfirstlane(s_ax[0].o0[l]);
        const int ox1 = __builtin_amdgcn_readfirstlane(s_ax[0].o1[l]);
        const int oy0 = __builtin_amdgcn_readfirstlane(s_ax[1].o0[l]);
        const int oy1 = __builtin_amdgcn_readfirstlane(s_ax[1].o1[l]);
        const uint8_t *sb = pool + (((l - 1) & 1) ? it.odd_off : 0);
        uint8_t *db = pool + ((l & 1) ? it.odd_off : 0);
        const int dst_stride = cw + 4;
        const int nq = cw >> 2;
        const int qlog = nq > 32 ? 6 : nq > 16 ? 5 : nq > 8 ? 4 : 3;
        const int QL = 1 << qlog, groups = 256 >> qlog;
        const int g = tid >> qlog, ql = tid & (QL - 1);
        const int R = (ch + groups - 1) / groups;
        const int r0 = g * R, r1 = min(ch, r0 + R);
        uint8_t *gout = pyr + s_off[l];
        const int gpitch = s_pitch[l];
        for (int q = ql; q < nq; q += QL) {
            const uint4 ex = *(const uint4 *)(s_tab + xoff + 4 * q);
            const int o0 = (int)(ex.x & 0xFFFFu), o1 = (int)(ex.y & 0xFFFFu);
            const int o2 = (int)(ex.z & 0xFFFFu), o3 = (int)(ex.w & 0xFFFFu);
            const int base01 = o0 & ~3, base23 = o2 & ~3;
            const uint32_t selA01 = (uint32_t)(o0 - base01) | 0x0C00u | ((uint32_t)(o1 - base01) << 16) | 0x0C000000u;
            const uint32_t selA23 = (uint32_t)(o2 - base23) | 0x0C00u | ((uint32_t)(o3 - base23) << 16) | 0x0C000000u;
            const uint32_t selB01 = selA01 + 0x00010001u, selB23 = selA23 + 0x00010001u;
            const pu2 W01 = {(unsigned short)(256 - (ex.x >> 16)), (unsigned short)(256 - (ex.y >> 16))};
            const pu2 W23 = {(unsigned short)(256 - (ex.z >> 16)), (unsigned short)(256 - (ex.w >> 16))};
            const pu2 F01 = {(unsigned short)(ex.x >> 16), (unsigned short)(ex.y >> 16)};
            const pu2 F23 = {(unsigned short)(ex.z >> 16), (unsigned short)(ex.w >> 16)};
            auto hrow = [&](int ya, pu2 &h01, pu2 &h23) {
                const uint8_t *r = sb + ya * src_stride;
                const uint32_t d0 = *(const uint32_t *)(r + base01), d1 = *(const uint32_t *)(r + base01 + 4);
                const uint32_t e0 = *(const uint32_t *)(r + base23), e1 = *(const uint32_t *)(r + base23 + 4);
                const pu2 A01 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(d1, d0, selA01));
                const pu2 B01 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(d1, d0, selB01));
                const pu2 A23 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(e1, e0, selA23));
                const pu2 B23 = __builtin_bit_cast(pu2, __builtin_amdgcn_perm(e1, e0, selB23));
                h01 = A01 * W01 + B01 * F01;
                h23 = A23 * W23 + B23 * F23;
            };
            const int gx = cx0 + 4 * q;
            const bool own_x = gx >= ox0 && gx < ox1;
            const int nbytes = min(4, ox1 - gx);
            int cur = -2;
            pu2 t01, t23, u01, u23;
            for (int r = r0; r < r1; r++) {
                const uint32_t e = s_tab[yoff + r];
                const int ya = (int)(e & 0xFFFFu);
                const uint32_t fy = e >> 16, wf = (256u - fy) | (fy << 16);
                if (ya == cur + 1) {
                    t01 = u01;
                    t23 = u23;
                    hrow(ya + 1, u01, u23);
                } else if (ya != cur) {
                    hrow(ya, t01, t23);
                    hrow(ya + 1, u01, u23);
                }
                cur = ya;
                const uint32_t word = vlerp4(t01, t23, u01, u23, wf);
                *(uint32_t *)(db + r * dst_stride + 4 * q) = word;
                const int gy = cy0 + r;
                if (own_x && gy >= oy0 && gy < oy1) {
                    uint8_t *o = gout + (int64_t)gy * gpitch + gx;
                    if (nbytes == 4) {
                        *(uint32_t *)o = word;
                    } else {
                        for (int j = 0; j < nbytes; j++) o[j] = (uint8_t)(word >> (8 * j));
                    }
                }
            }
        }
        xoff += cw;
        yoff += ch;
        src_stride = dst_stride;
    }
}

// ---------------------------------------------------------------- planning

// Plans of one axis of one image size: n[l] = level sizes, tab[l] = first
// resampling table entry of level l >= 1 in `coord`.  quad = 4 (columns:
// ranges in whole quads, level 0 in 16-byte chunks) or 1 (rows).
static void tower_axis(const std::vector<uint32_t> &coord, const int *n, const int *tab, int L, int nominal,
                       bool columns, std::vector<TowerAxis> *axes, std::vector<uint32_t> *ttab,
                       std::vector<int> *ax_tab, std::vector<int> *ax_ntab) {
    const int quad = columns ? 4 : 1, align0 = columns ? 16 : 1;
    auto A = [&](int l, int o) { return (int)(coord[tab[l] + o] & 0xFFFFu); };
    auto up = [](int v, int m) { return (v + m - 1) / m * m; };
    const int units = (n[1] + quad - 1) / quad;
    const int k = std::min(units, std::max(1, (n[1] + nominal - 1) / nominal));
    std::vector<std::vector<int>> bnd(L, std::vector<int>(k + 1, 0));
    for (int j = 0; j <= k; j++) bnd[1][j] = std::min(n[1], quad * (int)((int64_t)j * units / k));
    for (int l = 2; l < L; l++) {
        int o = 0;
        for (int j = 0; j <= k; j++) {
            // first output of level l whose source lies at or after the
            // boundary of level l - 1 (monotone in j: one sweep)
            while (o < n[l] && A(l, o) < bnd[l - 1][j]) o++;
            bnd[l][j] = std::min(n[l], up(o, quad));
        }
        bnd[l][0] = 0;
        bnd[l][k] = n[l];
    }
    for (int j = 0; j < k; j++) {
        std::vector<int> c0(L), c1(L);
        c0[L - 1] = bnd[L - 1][j];
        c1[L - 1] = bnd[L - 1][j + 1] > c0[L - 1] ? up(bnd[L - 1][j + 1], quad) : c0[L - 1];
        for (int l = L - 1; l >= 2; l--) {
            int lo = bnd[l - 1][j], hi = bnd[l - 1][j + 1];
            if (c1[l] > c0[l]) {
                const int alo = A(l, std::min(c0[l], n[l] - 1));
                const int ahi = std::min(A(l, std::min(c1[l] - 1, n[l] - 1)) + 1, n[l - 1] - 1);
                if (lo >= hi) {
                    lo = alo;
                    hi = ahi + 1;
                } else {
                    lo = std::min(lo, alo);
                    hi = std::max(hi, ahi + 1);
                }
            }
            if (lo < hi) {
                lo = lo / quad * quad;
                hi = up(hi, quad);
            } else {
                hi = lo;
            }
            c0[l - 1] = lo;
            c1[l - 1] = hi;
        }
        {
            const int alo = A(1, std::min(c0[1], n[1] - 1));
            const int ahi = std::min(A(1, std::min(c1[1] - 1, n[1] - 1)) + 1, n[0] - 1);
            c0[0] = alo / align0 * align0;
            c1[0] = columns ? c0[0] + up(ahi + 1 - c0[0], align0) : ahi + 1;
        }
        TowerAxis ax{};
        for (int l = 0; l < L; l++) {
            ax.c0[l] = (int16_t)c0[l];
            ax.cn[l] = (int16_t)(c1[l] - c0[l]);
            if (l >= 1) {
                ax.o0[l] = (int16_t)bnd[l][j];
                ax.o1[l] = (int16_t)bnd[l][j + 1];
            }
        }
        ax_tab->push_back((int)ttab->size());
        for (int l = 1; l < L; l++)
            for (int c = c0[l]; c < c1[l]; c++) {
                const uint32_t e = coord[tab[l] + std::min(c, n[l] - 1)];
                ttab->push_back(((e & 0xFFFFu) - (uint32_t)c0[l - 1]) | (e & 0xFFFF0000u));
            }
        ax_ntab->push_back((int)ttab->size() - ax_tab->back());
        axes->push_back(ax);
    }
}

bool tower_plan(vsfe_batch *b, int tw, int th) {
    b->h_twr_axes.clear();
    b->h_twr_tab.clear();
    b->h_twr_items.clear();
    b->twr_tw = tw;
    b->twr_th = th;
    b->twr_tab_cap = 0;
    b->twr_lds = 0;
    const int L = b->info.n_levels;
    if (L < 2) return true;
    std::vector<int> ax_tab, ax_ntab;
    struct Size { int w, h, x_first, x_count, y_first, y_count; };
    std::vector<Size> sizes;
    int tab_cap = 0, lds = 0;
    for (int i = 0; i < b->n_images; i++) {
        const ImageDev &im = b->images[i];
        int si = -1;
        for (int s = 0; s < (int)sizes.size(); s++)
            if (sizes[s].w == im.w && sizes[s].h == im.h) si = s;
        if (si < 0) {
            int nx[VSFE_MAX_LEVELS], ny[VSFE_MAX_LEVELS], tx[VSFE_MAX_LEVELS], ty[VSFE_MAX_LEVELS];
            for (int l = 0; l < L; l++) {
                nx[l] = im.lv[l].w;
                ny[l] = im.lv[l].h;
                tx[l] = im.lv[l].xtab;
                ty[l] = im.lv[l].ytab;
            }
            Size sz{im.w, im.h, (int)b->h_twr_axes.size(), 0, 0, 0};
            tower_axis(b->h_coord, nx, tx, L, tw, true, &b->h_twr_axes, &b->h_twr_tab, &ax_tab, &ax_ntab);
            sz.x_count = (int)b->h_twr_axes.size() - sz.x_first;
            sz.y_first = (int)b->h_twr_axes.size();
            tower_axis(b->h_coord, ny, ty, L, th, false, &b->h_twr_axes, &b->h_twr_tab, &ax_tab, &ax_ntab);
            sz.y_count = (int)b->h_twr_axes.size() - sz.y_first;
            si = (int)sizes.size();
            sizes.push_back(sz);
        }
        const Size &sz = sizes[si];
        for (int ay = sz.y_first; ay < sz.y_first + sz.y_count; ay++)
            for (int ax = sz.x_first; ax < sz.x_first + sz.x_count; ax++) {
                const TowerAxis &X = b->h_twr_axes[ax], &Y = b->h_twr_axes[ay];
                TowerItem t{};
                t.src_offset = im.lv[0].offset;
                t.sw = im.lv[0].w;
                t.sh = im.lv[0].h;
                t.spitch = im.lv[0].pitch;
                t.xs = X.c0[0];
                t.ncols = X.cn[0];
                t.ys = Y.c0[0];
                t.nrows = Y.cn[0];
                t.image = i;
                t.ax = ax;
                t.ay = ay;
                t.tabx = ax_tab[ax];
                t.ntabx = ax_ntab[ax];
                t.taby = ax_tab[ay];
                t.ntaby = ax_ntab[ay];
                // level buffers: level 0 with 16 padding columns, the others
                // with 4; one padding row each
                int even = 0, odd = 0;
                for (int l = 0; l < L; l++) {
                    const int bytes = (l == 0 ? X.cn[0] + 16 : X.cn[l] + 4) * (Y.cn[l] + 1);
                    if (l & 1) odd = std::max(odd, bytes);
                    else even = std::max(even, bytes);
                }
                t.odd_off = (even + 15) & ~15;
                if ((X.cn[0] >> 4) * Y.cn[0] > 256 * TWR_STAGE) return false;
                if (t.ntabx + t.ntaby > TWR_TAB) return false;
                tab_cap = std::max(tab_cap, (t.ntabx + t.ntaby + 3) & ~3);
                lds = std::max(lds, t.odd_off + odd);
                b->h_twr_items.push_back(t);
            }
    }
    b->twr_tab_cap = tab_cap;
    b->twr_lds = tab_cap * 4 + lds;
    return b->twr_lds <= TWR_LDS;
}

void tower_release(vsfe_batch *b) {
    if (b->d_twr_axes) (void)hipFree(b->d_twr_axes);
    if (b->d_twr_tab) (void)hipFree(b->d_twr_tab);
    if (b->d_twr_items) (void)hipFree(b->d_twr_items);
    b->d_twr_axes = nullptr;
    b->d_twr_tab = nullptr;
    b->d_twr_items = nullptr;
}

template <class T>
static int32_t tower_put(const std::vector<T> &v, T **dst) {
    if (v.empty()) return VSFE_OK;
    if (hipMalloc((void **)dst, v.size() * sizeof(T)) != hipSuccess)
        return fail(VSFE_EHIP, "hipMalloc of a pyramid plan table failed");
    if (hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return fail(VSFE_EHIP, "upload of a pyramid plan table failed");
    return VSFE_OK;
}

int32_t tower_upload(vsfe_batch *b) {
    tower_release(b);
    int32_t rc = tower_put(b->h_twr_axes, &b->d_twr_axes);
    if (!rc) rc = tower_put(b->h_twr_tab, &b->d_twr_tab);
    if (!rc) rc = tower_put(b->h_twr_items, &b->d_twr_items);
    return rc;
}

}  // namespace vsfe

using namespace vsfe;

int32_t vsfe::pyr_schedule_resolved(const vsfe_batch *b) {
    if (!b->twr_ok || b->info.n_levels < 2) return VSFE_PYR_LEVELS;
    if (b->pyr_schedule == VSFE_PYR_AUTO) {
        int64_t px = 0;
        for (const ImageDev &im : b->images) px += (int64_t)im.w * im.h;
        return px <= TWR_AUTO_PIXELS ? VSFE_PYR_TOWER : VSFE_PYR_LEVELS;
    }
    return b->pyr_schedule;
}

static int32_t build_range(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images, uint8_t *pyr,
                           int32_t *status, int lb, int le, bool whole, hipStream_t st) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!images || !pyr) return fail(VSFE_EINVAL, "null image or pyramid buffer");
    const int aligned = b->aligned_input16 && (((uintptr_t)images & 15) == 0) ? 1 : 0;
    if (whole && pyr_schedule_resolved(b) == VSFE_PYR_TOWER) {
        const int n = (int)b->h_twr_items.size();
        if (n <= 0) return VSFE_OK;
        hipLaunchKernelGGL(pyramid_tower_kernel, dim3(n), dim3(256), (size_t)b->twr_lds, st, b->d_images,
                           b->d_twr_items, b->d_twr_axes, b->d_twr_tab, b->info.n_levels, b->twr_tab_cap, images,
                           pyr, aligned);
        return check_launch("pyramid_build");
    }
    for (int l = lb; l < le; l++) {
        const int n = b->pyr_start[l + 1] - b->pyr_start[l];
        if (n <= 0) continue;
        hipLaunchKernelGGL(pyramid_level_kernel, dim3(n), dim3(256), 0, st, b->d_images,
                           b->d_pyr_items + b->pyr_start[l], l, b->d_coord, images, pyr, aligned);
        rc = check_launch("pyramid_build");
        if (rc) return rc;
    }
    return VSFE_OK;
}

extern "C" int32_t pyramid_build(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                 uint8_t *pyr, int32_t *status, void *stream) {
    if (!b) return fail(VSFE_EINVAL, "null batch");
    return build_range(ctx, b, images, pyr, status, 1, b->info.n_levels, true, (hipStream_t)stream);
}

extern "C" int32_t pyramid_build_levels(const vsfe_ctx *ctx, const vsfe_batch *b, const uint8_t *images,
                                        uint8_t *pyr, int32_t level_begin, int32_t level_end, int32_t *status,
                                        void *stream) {
    if (!b) return fail(VSFE_EINVAL, "null batch");
    if (level_begin < 1 || level_end > b->info.n_levels || level_begin >= level_end)
        return fail(VSFE_EINVAL, "level range out of 1..n_levels or empty");
    return build_range(ctx, b, images, pyr, status, level_begin, level_end, false, (hipStream_t)stream);
}

extern "C" int32_t vsfe_batch_set_pyramid(vsfe_batch *b, int32_t schedule, int32_t tile_w, int32_t tile_h) {
    if (!b) return fail(VSFE_EINVAL, "null batch");
    if (schedule != VSFE_PYR_AUTO && schedule != VSFE_PYR_LEVELS && schedule != VSFE_PYR_TOWER)
        return fail(VSFE_EINVAL, "unknown pyramid schedule");
    if (tile_w == 0) tile_w = b->twr_def_w;
    if (tile_h == 0) tile_h = b->twr_def_h;
    if (tile_w < 16 || tile_w > 240 || (tile_w & 3) || tile_h < 4 || tile_h > 64)
        return fail(VSFE_EINVAL, "tile out of range (16..240 columns, a multiple of 4; 4..64 rows)");
    if (tile_w != b->twr_tw || tile_h != b->twr_th) {
        // the device tables may still be read by queued launches
        if (hipDeviceSynchronize() != hipSuccess) return fail(VSFE_EHIP, "device synchronisation failed");
        if (!tower_plan(b, tile_w, tile_h)) {
            b->twr_ok = tower_plan(b, b->twr_def_w, b->twr_def_h);
            const int32_t rc = b->twr_ok ? tower_upload(b) : (tower_release(b), VSFE_OK);
            if (rc) {
                b->twr_ok = false;
                return rc;
            }
            return fail(VSFE_ECAPACITY, "a single-launch block of this tile exceeds its LDS or staging limits");
        }
        b->twr_ok = true;
        const int32_t rc = tower_upload(b);
        if (rc) {
            b->twr_ok = false;
            return rc;
        }
    }
    if (schedule == VSFE_PYR_TOWER && !b->twr_ok)
        return fail(VSFE_ECAPACITY, "the single-launch schedule is unavailable for this batch");
    b->pyr_schedule = schedule;
    return VSFE_OK;
}

extern "C" int32_t vsfe_batch_pyramid_get(const vsfe_batch *b, int32_t *schedule, int32_t *tile_w, int32_t *tile_h) {
    if (!b || !schedule || !tile_w || !tile_h) return fail(VSFE_EINVAL, "null argument");
    *schedule = pyr_schedule_resolved(b);
    *tile_w = b->twr_tw;
    *tile_h = b->twr_th;
    return VSFE_OK;
}
