// Pyramidal Feature Aggregation and the keypoint cap (Sec. II-C-2).
//
// The paper projects every culled keypoint to the native scale, writes the
// responses into a dense zero-initialised M[N_s][H][W], sums it into K_r
// and K_l, and runs a sparse q x q NMS around keypoints.  A dense M costs
// more HBM bytes than the pyramid itself, so here the same quantities are
// gathered sparsely: a native-scale position can only receive, from level
// m, the keypoint of one of the few level-m cells whose pixels project into
// the (2r+1)^2 window, so each keypoint reads those cells' keys (L2
// resident) and accumulates K_l / K_r for every window position.  The sums
// are integers, so the result equals the dense formulation exactly.
//
// Kernel 1 (one thread per cell): rank = (K_l << 16) | K_r of surviving
//   keypoints, 0 for empty or suppressed cells.
// Kernel 2 (one block per image): if more than n_max survive, a two-pass
//   radix select finds the n_max-th largest rank T; cells with rank > T and
//   the first (in canonical order) cells with rank == T are kept; a block
//   prefix sum compacts the survivors into the keypoint arrays in canonical
//   order (level, cell row, cell column).
#include <string.h>

#include <mutex>

#include "vsfe_internal.h"

namespace vsfe {

// Scratch of the allocation-free entry point pyca_cull_aggregate_noalloc:
// one uint32 rank per cell, at most VSFE_NOALLOC_MAX_CELLS cells (16 MiB).
// Each GPU the library runs on holds its own copy for the life of the
// process.  In host code `scratch` names a host-side stand-in, never the
// device array: its device address is looked up once per device
// (pyca_prepare, at context creation) and only that address is passed on.
static __device__ __align__(256) uint32_t scratch[VSFE_NOALLOC_MAX_CELLS];
constexpr int SCRATCH_DEVICES = 64;
static uint32_t *g_scratch_ptr[SCRATCH_DEVICES];
static std::mutex g_scratch_mu;

int32_t pyca_prepare(int device) {
    if (device < 0 || device >= SCRATCH_DEVICES) return fail(VSFE_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return VSFE_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(VSFE_EHIP, std::string("address of the aggregation scratch: ") + hipGetErrorString(e));
    g_scratch_ptr[device] = (uint32_t *)ptr;
    return VSFE_OK;
}

// x * S approximates the native coordinate times 2^16 (x < 8192 / 1.2^l,
// S < 65536 * 1.2^l + 1), so it stays below 2^29: a 24-bit multiply.
__device__ __forceinline__ int project_q16(int x, int S, int limit) {
    const int v = (int)((__umul24((uint32_t)x, (uint32_t)S) + 32768u) >> 16);
    return v < limit - 1 ? v : limit - 1;
}

// FIX2: the host has checked that at every level the window touches at most
// 2 x 2 cells, so all candidate keys are loaded up front (all levels' loads
// in flight together) and then accumulated; otherwise cells are visited in
// a loop per level.
//
// A native position receives at most one keypoint per level (projection
// scales up, so distinct level pixels land on distinct native pixels), so
// K_l <= 8 and K_r <= 8 * 4095 < 2^15: the pair is kept packed as
// (K_l << 16) | K_r, which is also the rank and orders lexicographically.
// Divisions by a level's cell size use a per-level reciprocal,
// floor(x / c) = (x * (floor(2^20 / c) + 1)) >> 20, exact for 0 <= x < 8192
// (the largest image side) and c <= 128 (the error, below x / 2^20 < 1/128,
// stays under 1 / c); cells are at most 32 pixels.
// Per-level constants of the aggregation, the same for every image of a
// batch (level scale and cell side come from the parameters): 1 / scale
// and ceil(2^20 / cell), the multiplier that divides offsets below 1024 by
// the cell side exactly.
struct PfaLevelTab {
    float inv[VSFE_MAX_LEVELS];
    uint32_t mag[VSFE_MAX_LEVELS];
};

template <int R, bool FIX2>
__global__ __launch_bounds__(256) void pfa_eval_kernel(const ImageDev *__restrict__ imgs,
                                                       const CellChunk *__restrict__ chunks,
                                                       const uint32_t *__restrict__ cell_keys,
                                                       uint32_t *__restrict__ rank, int pfa, int nms_mode,
                                                       PfaLevelTab tab) {
    constexpr int Q = 2 * R + 1, NS = Q * Q, CENTER = R * Q + R;
    __shared__ uint32_t s_acc[NS][256];     // each thread's window sums (thread-private columns)
    const float *s_inv = tab.inv;           // per level, the same for every image of the batch
    const uint32_t *s_mag = tab.mag;
    const CellChunk ch = chunks[xcd_item(blockIdx.x, gridDim.x)];
    const ImageDev &im = imgs[ch.image];
    const LevelDev lv = im.lv[ch.level];
    const int idx = (int)ch.first + (int)threadIdx.x;
    if (idx >= lv.ncx * lv.ncy) return;
    const int64_t g = lv.cell_offset + idx;
    const uint32_t key = cell_keys[g];
    if (!key) {
        rank[g] = 0;
        return;
    }
    const int c = lv.cell, cy = idx / lv.ncx, cx = idx - cy * lv.ncx;
    const int off = 1023 - (int)(key & 1023u);
    const int oy = (int)(__umul24((uint32_t)off, s_mag[ch.level]) >> 20);
    const int x = cx * c + (off - oy * c), y = cy * c + oy;
    const int score = (int)((key >> 10) & 0xFFFu);
    if (!pfa) {
        rank[g] = (1u << 16) | (uint32_t)score;
        return;
    }
    const int px = project_q16(x, lv.scale_q16, im.w), py = project_q16(y, lv.scale_q16, im.h);
    // the window sums live in LDS: a hit is one LDS add, not a select over
    // every window position
    const int tid = threadIdx.x;
#pragma unroll
    for (int s = 0; s < NS; s++) s_acc[s][tid] = 0;
    // candidate cells of level m: those whose pixels can project into the window
    auto window = [&](int m, const LevelDev &L, int *a0, int *a1, int *b0, int *b1) {
        const float inv = s_inv[m];
        int xlo = (int)floorf(((float)(px - R) - 0.5f) * inv) - 1, xhi = (int)floorf(((float)(px + R) + 0.5f) * inv) + 1;
        int ylo = (int)floorf(((float)(py - R) - 0.5f) * inv) - 1, yhi = (int)floorf(((float)(py + R) + 0.5f) * inv) + 1;
        xlo = max(xlo, 0);
        ylo = max(ylo, 0);
        xhi = min(xhi, L.w - 1);
        yhi = min(yhi, L.h - 1);
        if (xlo > xhi || ylo > yhi) return false;
        const uint32_t mag = s_mag[m];
        *a0 = (int)(__umul24((uint32_t)xlo, mag) >> 20);
        *a1 = (int)(__umul24((uint32_t)xhi, mag) >> 20);
        *b0 = (int)(__umul24((uint32_t)ylo, mag) >> 20);
        *b1 = (int)(__umul24((uint32_t)yhi, mag) >> 20);
        return true;
    };
    auto add = [&](int m, const LevelDev &L, int aa, int bb, uint32_t k) {
        if (!k) return;
        const int cm = L.cell;
        const int o = 1023 - (int)(k & 1023u);
        const int orow = (int)(__umul24((uint32_t)o, s_mag[m]) >> 20);
        const int qx = project_q16(__umul24(aa, cm) + (o - __umul24(orow, cm)), L.scale_q16, im.w) - px;
        const int qy = project_q16(__umul24(bb, cm) + orow, L.scale_q16, im.h) - py;
        if (qx < -R || qx > R || qy < -R || qy > R) return;
        const int slot = (qy + R) * Q + (qx + R);
        atomicAdd(&s_acc[slot][tid], (1u << 16) | ((k >> 10) & 0xFFFu));
    };
    if constexpr (FIX2) {
        uint32_t kk[VSFE_MAX_LEVELS][4];
        int ca[VSFE_MAX_LEVELS], cb[VSFE_MAX_LEVELS];
#pragma unroll
        for (int m = 0; m < VSFE_MAX_LEVELS; m++) {
            kk[m][0] = kk[m][1] = kk[m][2] = kk[m][3] = 0u;
            ca[m] = cb[m] = 0;
            if (m < im.n_levels) {
                const LevelDev L = im.lv[m];
                int a0, a1, b0, b1;
                if (window(m, L, &a0, &a1, &b0, &b1)) {
                    ca[m] = a0;
                    cb[m] = b0;
                    // 32-bit byte offsets from the level's uniform base (a
                    // level holds fewer than 2^24 cells), so each load is
                    // one vector offset on a scalar address
                    typedef const __attribute__((address_space(1))) uint8_t gbyte;
                    typedef const __attribute__((address_space(1))) uint32_t gword;
                    gbyte *kb = (gbyte *)(cell_keys + L.cell_offset);
                    const uint32_t o0 = 4u * (__umul24((uint32_t)b0, (uint32_t)L.ncx) + (uint32_t)a0);
                    const uint32_t rowb = 4u * (uint32_t)L.ncx;
                    const bool ax = a0 + 1 < L.ncx, by = b0 + 1 < L.ncy;
                    kk[m][0] = *(gword *)(kb + o0);
                    if (ax) kk[m][1] = *(gword *)(kb + (o0 + 4u));
                    if (by) kk[m][2] = *(gword *)(kb + (o0 + rowb));
                    if (ax && by) kk[m][3] = *(gword *)(kb + (o0 + rowb + 4u));
                }
            }
        }
#pragma unroll
        for (int m = 0; m < VSFE_MAX_LEVELS; m++) {
            if (m < im.n_levels) {
                const LevelDev L = im.lv[m];
#pragma unroll
                for (int q = 0; q < 4; q++) add(m, L, ca[m] + (q & 1), cb[m] + (q >> 1), kk[m][q]);
            }
        }
    } else {
        for (int m = 0; m < im.n_levels; m++) {
            const LevelDev L = im.lv[m];
            int a0, a1, b0, b1;
            if (!window(m, L, &a0, &a1, &b0, &b1)) continue;
            a1 = min(a1, L.ncx - 1);
            b1 = min(b1, L.ncy - 1);
            for (int bb = b0; bb <= b1; bb++)
                for (int aa = a0; aa <= a1; aa++) add(m, L, aa, bb, cell_keys[L.cell_offset + (int64_t)bb * L.ncx + aa]);
        }
    }
    const uint32_t own = s_acc[CENTER][tid];
    bool sup = false;
#pragma unroll
    for (int s = 0; s < NS; s++) {
        const uint32_t a = s_acc[s][tid];
        if (s == CENTER || a == 0) continue;
        // mode 0: (K_l, K_r) lexicographically larger; mode 1: both larger
        sup = sup || (nms_mode == 0 ? a > own : ((a >> 16) > (own >> 16) && (a & 0xFFFFu) > (own & 0xFFFFu)));
    }
    rank[g] = sup ? 0u : own;
}

constexpr int SEL_THREADS = 1024;
constexpr int SEL_WAVES = SEL_THREADS / 64;
constexpr int SEL_LDS_CELLS = 24576;      // an image's ranks are cached in LDS up to this many cells
constexpr int SEL_CHUNK = 8;              // cells per thread whose rank and key are read together
constexpr int SEL_IDX_SLOTS = 8192;       // keypoints per image written out slot by slot (beyond: cell by cell)

// Exclusive prefix sums of two per-thread counts over the block; *tot_a /
// *tot_b get the totals.  Two barriers: every thread must call it.
__device__ __forceinline__ void block_scan2(int a, int b, int *wave_a, int *wave_b, int *ex_a, int *ex_b, int *tot_a,
                                            int *tot_b) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int ia = a, ib = b;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int va = __shfl_up(ia, d), vb = __shfl_up(ib, d);
        if (lane >= d) {
            ia += va;
            ib += vb;
        }
    }
    if (lane == 63) {
        wave_a[wave] = ia;
        wave_b[wave] = ib;
    }
    __syncthreads();
    int ba = 0, bb = 0, ta = 0, tb = 0;
    for (int w = 0; w < SEL_WAVES; w++) {
        const int xa = wave_a[w], xb = wave_b[w];
        ba += w < wave ? xa : 0;
        bb += w < wave ? xb : 0;
        ta += xa;
        tb += xb;
    }
    __syncthreads();
    *ex_a = ba + ia - a;
    *ex_b = bb + ib - b;
    *tot_a = ta;
    *tot_b = tb;
}

// Over the 1024 buckets of hist, from the top: the bucket where the running
// count (starting at base) first reaches need.  Thread t takes bucket
// 1023 - t; a block scan of the counts finds the crossing thread.  Writes
// the bucket to s_sel[slot_bkt] and the count above it to s_sel[slot_acc].
// Every thread must call it (two barriers).
__device__ __forceinline__ void find_bucket(const int *hist, int base, int need, int *wave_cnt, int *s_sel,
                                            int slot_bkt, int slot_acc) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = hist[1023 - tid];
    int incl = h;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    if (lane == 63) wave_cnt[wave] = incl;
    __syncthreads();
    int before = base;
    for (int w = 0; w < wave; w++) before += wave_cnt[w];
    incl += before;
    // the crossing thread: running count before it < need <= running count with it
    if (incl >= need && incl - h < need) {
        s_sel[slot_bkt] = 1023 - tid;
        s_sel[slot_acc] = incl - h;
    }
    __syncthreads();
}

// One block per image.  The image's ranks are read once (into LDS when
// they fit); the compaction gives each thread a contiguous run of cells, so
// one block scan of the per-thread counts places every survivor.  Up to
// SEL_IDX_SLOTS survivors, the threads first record the cell of every slot
// in LDS and then write the keypoints one slot per thread (coalesced);
// beyond that, each thread writes its own cells' keypoints.
__global__ __launch_bounds__(SEL_THREADS) void select_compact_kernel(
    const ImageDev *__restrict__ imgs, const uint32_t *__restrict__ cell_keys, const uint32_t *__restrict__ rank,
    vsfe_kp_soa kps, int32_t *__restrict__ kp_count, int n_max, int32_t *status, PfaLevelTab tab) {
    __shared__ uint32_t s_rank[SEL_LDS_CELLS];
    __shared__ int hist[1024];
    __shared__ int wave_a[SEL_WAVES], wave_b[SEL_WAVES];
    __shared__ int s_sel[3];   // threshold T, count of ranks > T, bucket
    // the image's level records as the compaction reads them (first cell
    // relative to the image, cells per row, cell size, scale, offset divisor)
    __shared__ int4 s_lv[VSFE_MAX_LEVELS];
    __shared__ uint32_t s_mag[VSFE_MAX_LEVELS];
    __shared__ int s_idx[SEL_IDX_SLOTS];      // slot -> cell of the image
    const ImageDev &im = imgs[blockIdx.x];
    const int64_t base = im.cell_base;
    const int n = (int)im.n_cells;
    const int n_levels = im.n_levels, W = im.w, H = im.h;
    const int64_t kp0 = im.kp_offset;
    const int tid = threadIdx.x;
    const bool cached = n <= SEL_LDS_CELLS;
    auto rk = [&](int i) { return cached ? s_rank[i] : rank[base + i]; };
    if (tid < n_levels) {
        const LevelDev &L = im.lv[tid];
        s_lv[tid] = make_int4((int)(L.cell_offset - base), L.ncx, L.cell, L.scale_q16);
        s_mag[tid] = tab.mag[tid];
    }

    // pass 1: histogram of the high 10 bits of the nonzero ranks (ranks <
    // 2^20); its total is the number of survivors.  Four loads per thread
    // are in flight at once.
    hist[tid] = 0;
    __syncthreads();
    for (int i0 = 0; i0 < n; i0 += 4 * SEL_THREADS) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int i = i0 + u * SEL_THREADS + tid;
            v[u] = i < n ? rank[base + i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int i = i0 + u * SEL_THREADS + tid;
            if (cached && i < n) s_rank[i] = v[u];
            if (v[u]) atomicAdd(&hist[v[u] >> 10], 1);
        }
    }
    __syncthreads();
    {
        const int lane = tid & 63, wave = tid >> 6;
        int v = hist[tid];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) wave_a[wave] = v;
    }
    __syncthreads();
    int m = 0;
    for (int w = 0; w < SEL_WAVES; w++) m += wave_a[w];

    uint32_t T = 0;
    int quota = 0;
    if (m > n_max) {
        // bucket of the n_max-th largest rank, then its low 10 bits
        find_bucket(hist, 0, n_max, wave_a, s_sel, 2, 1);
        const int bucket = s_sel[2];
        hist[tid] = 0;
        __syncthreads();
        for (int i = tid; i < n; i += SEL_THREADS) {
            const uint32_t v = rk(i);
            if (v && (int)(v >> 10) == bucket) atomicAdd(&hist[v & 1023u], 1);
        }
        __syncthreads();
        find_bucket(hist, s_sel[1], n_max, wave_a, s_sel, 0, 1);
        T = (uint32_t)((bucket << 10) | s_sel[0]);
        quota = n_max - s_sel[1];
    }

    // compaction in canonical order: thread t owns cells [t seg, (t+1) seg);
    // a cell's slot is (# ranks above T before it) + min(# equal to T before
    // it, quota)
    const int seg = (n + SEL_THREADS - 1) / SEL_THREADS;
    const int i0 = min(n, tid * seg), i1 = min(n, i0 + seg);
    int n_gt = 0, n_eq = 0;
    for (int i = i0; i < i1; i++) {
        const uint32_t v = rk(i);
        n_gt += (v != 0 && v > T) ? 1 : 0;
        n_eq += (v != 0 && T != 0 && v == T) ? 1 : 0;
    }
    int gt_before, eq_before, gt_all, eq_all;
    block_scan2(n_gt, n_eq, wave_a, wave_b, &gt_before, &eq_before, &gt_all, &eq_all);
    const int kept = gt_all + min(eq_all, quota);
    // keypoint stores through global pointers (they cannot touch the LDS
    // tables read between them)
    typedef __attribute__((address_space(1))) uint32_t g32;
    typedef __attribute__((address_space(1))) uint16_t g16;
    typedef __attribute__((address_space(1))) uint8_t g8;
    // (each array from the image's first slot: uniform bases, 32-bit slot offsets)
    g16 *const o_x = (g16 *)(kps.x + kp0), *const o_y = (g16 *)(kps.y + kp0);
    g16 *const o_score = (g16 *)(kps.score + kp0);
    g16 *const o_x0 = (g16 *)(kps.x0 + kp0), *const o_y0 = (g16 *)(kps.y0 + kp0);
    g32 *const o_kr = (g32 *)(kps.kr + kp0);
    g8 *const o_level = (g8 *)(kps.level + kp0), *const o_flags = (g8 *)(kps.flags + kp0);
    g8 *const o_kl = (g8 *)(kps.kl + kp0), *const o_bin = (g8 *)(kps.bin + kp0);
    // the keypoint of cell i (level l, rank v, key) into slot `slot`
    auto emit = [&](int i, int l, uint32_t v, uint32_t key, int slot) {
        const int4 lv = s_lv[l];                       // (first cell, ncx, cell, scale)
        const int li = i - lv.x;
        // li / ncx by a float reciprocal and one correction step (li <
        // 2^24, so the estimate is off by at most one); off / c by the
        // level's multiplier (off < 1024)
        const int c = lv.z;
        int cy = (int)((float)li * __builtin_amdgcn_rcpf((float)lv.y));
        int cx = li - cy * lv.y;
        if (cx < 0) { cy--; cx += lv.y; }
        if (cx >= lv.y) { cy++; cx -= lv.y; }
        const int off = 1023 - (int)(key & 1023u);
        const int oy = (int)(__umul24((uint32_t)off, s_mag[l]) >> 20);
        const int x = cx * c + (off - oy * c), y = cy * c + oy;
        // byte offsets computed in 32 bits (slot < 2^16), so each store is one
        // vector offset on a scalar base
        const uint32_t o = (uint32_t)slot;
        auto at2 = [&](g16 *a) { return (g16 *)((g8 *)a + 2u * o); };
        *at2(o_x) = (uint16_t)x;
        *at2(o_y) = (uint16_t)y;
        *(o_level + o) = (uint8_t)l;
        *(o_flags + o) = (key & VSFE_KEY_FALLBACK) ? (uint8_t)VSFE_KP_FALLBACK : (uint8_t)0;
        *at2(o_score) = (uint16_t)((key >> 10) & 0xFFFu);
        *at2(o_x0) = (uint16_t)project_q16(x, lv.w, W);
        *at2(o_y0) = (uint16_t)project_q16(y, lv.w, H);
        *(o_kl + o) = (uint8_t)(v >> 16);
        *(g32 *)((g8 *)o_kr + 4u * o) = v & 0xFFFFu;
        *(o_bin + o) = 0;
    };
    if (kept <= SEL_IDX_SLOTS && kept <= n_max) {                    // uniform
        // the slot -> cell map in LDS, then one thread per slot, so that
        // consecutive lanes write consecutive slots (full-width stores
        // instead of a narrow scattered store per field and kept cell)
        for (int c0 = i0; c0 < i1; c0 += SEL_CHUNK) {
            uint32_t vv[SEL_CHUNK];
#pragma unroll
            for (int u = 0; u < SEL_CHUNK; u++) vv[u] = c0 + u < i1 ? rk(c0 + u) : 0u;
#pragma unroll
            for (int u = 0; u < SEL_CHUNK; u++) {
                const uint32_t v = vv[u];                // (cells past i1 have v = 0)
                const bool gt = v != 0 && v > T;
                const bool eq = v != 0 && T != 0 && v == T;
                const bool keep = gt || (eq && eq_before < quota);
                if (keep) s_idx[gt_before + min(eq_before, quota)] = c0 + u;   // < kept
                gt_before += gt ? 1 : 0;
                eq_before += eq ? 1 : 0;
            }
        }
        __syncthreads();
        for (int slot = tid; slot < kept; slot += SEL_THREADS) {
            const int i = s_idx[slot];
            int l = 0;
            while (l + 1 < n_levels && s_lv[l + 1].x <= i) l++;
            emit(i, l, rk(i), cell_keys[base + i], slot);
        }
    } else {
        // each thread its own cells in chunks of SEL_CHUNK (ranks and keys of
        // a chunk read together)
        int l = 0;
        while (l + 1 < n_levels && s_lv[l + 1].x <= i0) l++;
        for (int c0 = i0; c0 < i1; c0 += SEL_CHUNK) {
            uint32_t vv[SEL_CHUNK], kk[SEL_CHUNK];
#pragma unroll
            for (int u = 0; u < SEL_CHUNK; u++) {
                const int i = c0 + u;
                vv[u] = i < i1 ? rk(i) : 0u;
                kk[u] = i < i1 ? cell_keys[base + i] : 0u;
            }
#pragma unroll
            for (int u = 0; u < SEL_CHUNK; u++) {
                const int i = c0 + u;
                const uint32_t v = vv[u];
                const bool gt = v != 0 && v > T;
                const bool eq = v != 0 && T != 0 && v == T;
                const bool keep = gt || (eq && eq_before < quota);
                const int slot = gt_before + min(eq_before, quota);
                gt_before += gt ? 1 : 0;
                eq_before += eq ? 1 : 0;
                if (!keep) continue;                       // (cells past i1 have v = 0)
                while (l + 1 < n_levels && s_lv[l + 1].x <= i) l++;
                if (slot < n_max) emit(i, l, v, kk[u], slot);
                else if (status) atomicOr(status, VSFE_DEV_OVERFLOW);
            }
        }
    }
    if (tid == 0) kp_count[blockIdx.x] = kept < n_max ? kept : n_max;
}

// Aggregation and cap with `rank` (one uint32 per cell of the batch) as
// the scratch: every cell's rank is written before it is read, so the
// scratch needs no clearing.
static int32_t pyca_run(const vsfe_ctx *ctx, const vsfe_batch *b, const uint32_t *cell_keys, uint32_t *rank,
                        const vsfe_kp_soa *kps, int32_t *kp_count, int32_t *status, hipStream_t st) {
    int32_t rc = VSFE_OK;
    const vsfe_params &p = ctx->p;
    PfaLevelTab tab;
    memset(&tab, 0, sizeof(tab));
    for (int l = 0; l < p.n_levels; l++) {
        tab.inv[l] = 65536.0f / (float)ctx->scale_q16[l];
        tab.mag[l] = (1u << 20) / (uint32_t)ctx->cell[l] + 1u;
    }
    if (b->n_chunks > 0) {
        // every level's window (at most (2r+1)/s + 4 pixels wide) within 2 x 2 cells?
        bool fix2 = true;
        for (int l = 0; l < p.n_levels; l++) {
            const double s_l = ctx->scale_q16[l] / 65536.0;
            if ((2 * p.nms_radius + 1) / s_l + 3.0 > (double)ctx->cell[l]) fix2 = false;
        }
#define VSFE_PFA_LAUNCH(R_)                                                                                       \
    do {                                                                                                          \
        if (fix2)                                                                                                 \
            hipLaunchKernelGGL((pfa_eval_kernel<R_, true>), dim3(b->n_chunks), dim3(256), 0, st, b->d_images,    \
                               b->d_chunks, cell_keys, rank, p.pfa, p.nms_mode, tab);                             \
        else                                                                                                      \
            hipLaunchKernelGGL((pfa_eval_kernel<R_, false>), dim3(b->n_chunks), dim3(256), 0, st, b->d_images,   \
                               b->d_chunks, cell_keys, rank, p.pfa, p.nms_mode, tab);                             \
    } while (0)
        switch (p.nms_radius) {
            case 0: VSFE_PFA_LAUNCH(0); break;
            case 1: VSFE_PFA_LAUNCH(1); break;
            case 2: VSFE_PFA_LAUNCH(2); break;
            default: VSFE_PFA_LAUNCH(3); break;
        }
#undef VSFE_PFA_LAUNCH
        rc = check_launch("pyca_cull_aggregate (aggregation)");
        if (rc) return rc;
    }
    hipLaunchKernelGGL(select_compact_kernel, dim3(b->n_images), dim3(SEL_THREADS), 0, st, b->d_images, cell_keys,
                       rank, *kps, kp_count, p.n_max, status, tab);
    return check_launch("pyca_cull_aggregate (select)");
}

static int32_t pyca_args(const vsfe_ctx *ctx, const vsfe_batch *b, const uint32_t *cell_keys, const vsfe_kp_soa *kps,
                         int32_t *kp_count, int32_t *status) {
    int32_t rc = check_common(ctx, b, status);
    if (rc) return rc;
    if (!cell_keys || !kps || !kp_count) return fail(VSFE_EINVAL, "null buffer");
    if (!kps->x || !kps->y || !kps->level || !kps->flags || !kps->score || !kps->x0 || !kps->y0 || !kps->kl ||
        !kps->kr || !kps->bin)
        return fail(VSFE_EINVAL, "null keypoint array");
    return VSFE_OK;
}

}  // namespace vsfe

using namespace vsfe;

extern "C" int32_t pyca_cull_aggregate(const vsfe_ctx *ctx, const vsfe_batch *b, const uint32_t *cell_keys,
                                       void *workspace, const vsfe_kp_soa *kps, int32_t *kp_count,
                                       int32_t *status, void *stream) {
    const int32_t rc = pyca_args(ctx, b, cell_keys, kps, kp_count, status);
    if (rc) return rc;
    if (!workspace) return fail(VSFE_EINVAL, "null workspace");
    return pyca_run(ctx, b, cell_keys, (uint32_t *)workspace, kps, kp_count, status, (hipStream_t)stream);
}

extern "C" int32_t pyca_cull_aggregate_noalloc(const vsfe_ctx *ctx, const vsfe_batch *b, const uint32_t *cell_keys,
                                               const vsfe_kp_soa *kps, int32_t *kp_count, int32_t *status,
                                               void *stream) {
    const int32_t rc = pyca_args(ctx, b, cell_keys, kps, kp_count, status);
    if (rc) return rc;
    if (b->info.n_cells > VSFE_NOALLOC_MAX_CELLS)
        return fail(VSFE_ECAPACITY, "batch has " + std::to_string(b->info.n_cells) +
                                        " cells; the allocation-free aggregation holds at most " +
                                        std::to_string((long long)VSFE_NOALLOC_MAX_CELLS));
    uint32_t *ptr = (ctx->device >= 0 && ctx->device < SCRATCH_DEVICES) ? g_scratch_ptr[ctx->device] : nullptr;
    if (!ptr) return fail(VSFE_EUNSUPPORTED, "aggregation scratch not prepared on this device");
    return pyca_run(ctx, b, cell_keys, ptr, kps, kp_count, status, (hipStream_t)stream);
}
