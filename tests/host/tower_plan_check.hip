// Host check of the single-launch pyramid schedule (test infrastructure):
// plans batches with the library's own planner, replays the kernel's reads
// and writes on the CPU (every LDS access bounds-checked, every weighted
// read checked to hit a byte written by the level above, every output pixel
// written exactly once) and compares the levels with the oracle pyramid.
// Built and run by tests/test_tower_plan_host.py.
#include "../../paper_2410_04090_amd/csrc/api.hip"
#include "../../paper_2410_04090_amd/csrc/pyramid.hip"
extern "C" {
#include "../../oracle/oracle.h"
}
#include <cstdio>
#include <random>
#include <cassert>

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { if (fails++ < 20) { printf("FAIL %s:%d ", __FILE__, __LINE__); printf(__VA_ARGS__); printf("\n"); } } } while (0)

static void run(int W, int H, int tw, int th, int L, unsigned seed) {
    vsfe_params p;
    vsfe_params_default(&p);
    p.n_levels = L;
    int32_t w[1] = {W}, h[1] = {H}, pitch[1] = {W + 3};
    int64_t off[1] = {0};
    vsfe_batch b;
    int rc = plan_batch(p, 128, 32, 1, w, h, pitch, off, &b);
    if (rc) { printf("plan_batch rc=%d for %dx%d L=%d\n", rc, W, H, L); return; }
    L = b.info.n_levels;
    bool ok = tower_plan(&b, tw, th);
    if (!ok) { printf("tower_plan: does not fit %dx%d tile %dx%d (lds %d)\n", W, H, tw, th, b.twr_lds); return; }
    std::mt19937 rng(seed);
    std::vector<uint8_t> img((size_t)pitch[0] * H);
    for (auto &v : img) v = rng() & 255;
    // oracle
    std::vector<uint8_t> ref((size_t)or_pyramid_bytes(W, H, L));
    or_pyramid(img.data(), W, H, pitch[0], L, ref.data());
    std::vector<int64_t> lbase(L, 0);
    for (int l = 1; l < L; l++) lbase[l] = lbase[l - 1] + (int64_t)b.images[0].lv[l - 1].w * b.images[0].lv[l - 1].h;
    // emulated output
    std::vector<std::vector<uint8_t>> out(L);
    std::vector<std::vector<int>> cnt(L);
    for (int l = 1; l < L; l++) {
        out[l].assign((size_t)b.images[0].lv[l].w * b.images[0].lv[l].h, 0);
        cnt[l].assign(out[l].size(), 0);
    }
    const int pool_size = b.twr_lds - 4 * b.twr_tab_cap;
    for (const TowerItem &it : b.h_twr_items) {
        const TowerAxis &X = b.h_twr_axes[it.ax], &Y = b.h_twr_axes[it.ay];
        std::vector<int> pool(pool_size, 0), tag(pool_size, -1);
        const int S0 = it.ncols + 16, cpr = it.ncols >> 4;
        CHECK(cpr * it.nrows <= 256 * TWR_STAGE, "staging tasks");
        CHECK(it.xs % 16 == 0 && it.ncols % 16 == 0, "alignment");
        for (int q = 0; q < 256 * TWR_STAGE; q++) {
            const int rr = q / cpr, k = q - rr * cpr;
            if (rr >= it.nrows) continue;
            const int gy = std::min(it.ys + rr, it.sh - 1);
            for (int j = 0; j < 16; j++) {
                const int gx = std::min(std::max(it.xs + 16 * k + j, 0), it.sw - 1);
                const int at = (rr * (S0 >> 4) + k) * 16 + j;
                CHECK(at >= 0 && at < it.odd_off, "staging store out of level-0 buffer %d", at);
                pool[at] = img[(size_t)gy * pitch[0] + gx];
                tag[at] = 0;
            }
        }
        std::vector<uint32_t> tab(b.twr_tab_cap, 0);
        CHECK(it.ntabx + it.ntaby <= b.twr_tab_cap, "table cap");
        for (int e = 0; e < it.ntabx + it.ntaby; e++)
            tab[e] = b.h_twr_tab[e < it.ntabx ? it.tabx + e : it.taby + (e - it.ntabx)];
        int xoff = 0, yoff = it.ntabx, src_stride = S0;
        for (int l = 1; l < L; l++) {
            const LevelDev &lv = b.images[0].lv[l];
            const int cw = X.cn[l], ch = Y.cn[l], cx0 = X.c0[l], cy0 = Y.c0[l];
            const int ox0 = X.o0[l], ox1 = X.o1[l], oy0 = Y.o0[l], oy1 = Y.o1[l];
            const int sbase = ((l - 1) & 1) ? it.odd_off : 0, dbase = (l & 1) ? it.odd_off : 0;
            const int src_rows = (l == 1 ? Y.cn[0] : Y.cn[l - 1]) + 1;
            const int src_end = sbase + src_stride * src_rows;
            const int dst_stride = cw + 4;
            CHECK(cw % 4 == 0, "cw quad");
            CHECK(xoff % 4 == 0, "xoff align");
            const int nq = cw >> 2;
            for (int q = 0; q < nq; q++) {
                uint32_t ex[4];
                for (int j = 0; j < 4; j++) ex[j] = tab[xoff + 4 * q + j];
                const int o0 = ex[0] & 0xFFFF, o2 = ex[2] & 0xFFFF;
                CHECK((o0 & ~3) + 7 < src_stride && (o2 & ~3) + 7 < src_stride, "dword reads past the row stride");
                for (int j = 0; j < 4; j++) {
                    const int oj = ex[j] & 0xFFFF;
                    CHECK(oj - (o0 & ~3) <= 6 || j >= 2, "selector range 01 %d", oj - (o0 & ~3));
                    if (j >= 2) CHECK(oj - (o2 & ~3) <= 6, "selector range 23");
                }
                for (int r = 0; r < ch; r++) {
                    const uint32_t e = tab[yoff + r];
                    const int ya = e & 0xFFFF, fy = e >> 16;
                    CHECK(sbase + (ya + 1) * src_stride + src_stride - 1 < src_end, "row beyond src buffer");
                    uint32_t word = 0;
                    for (int j = 0; j < 4; j++) {
                        const int oj = ex[j] & 0xFFFF, fx = ex[j] >> 16;
                        auto rd = [&](int yy, int xx, int wgt) {
                            const int at = sbase + yy * src_stride + xx;
                            CHECK(at >= 0 && at < pool_size, "read outside pool");
                            if (wgt) CHECK(tag[at] == l - 1, "weighted read of unwritten byte l=%d yy=%d xx=%d tag=%d", l, yy, xx, tag[at]);
                            return wgt ? pool[at] : 0;
                        };
                        const int64_t v = (int64_t)(256 - fx) * (256 - fy) * rd(ya, oj, 1) + (int64_t)fx * (256 - fy) * rd(ya, oj + 1, fx)
                                        + (int64_t)(256 - fx) * fy * rd(ya + 1, oj, fy) + (int64_t)fx * fy * rd(ya + 1, oj + 1, fx * fy);
                        const int px = (int)((v + 32768) >> 16);
                        word |= (uint32_t)px << (8 * j);
                        const int at = dbase + r * dst_stride + 4 * q + j;
                        CHECK(at >= 0 && at < pool_size, "write outside pool");
                        CHECK(l & 1 ? at >= it.odd_off : at + 0 < it.odd_off, "write into the other buffer");
                        pool[at] = px;
                        tag[at] = l;
                    }
                    const int gy = cy0 + r, gx = cx0 + 4 * q;
                    if (gx >= ox0 && gx < ox1 && gy >= oy0 && gy < oy1) {
                        const int nb = std::min(4, ox1 - gx);
                        CHECK(nb == 4 || ox1 == lv.w, "partial quad not at the right edge");
                        for (int j = 0; j < nb; j++) {
                            CHECK(gx + j < lv.w && gy < lv.h, "global write outside level");
                            if (gx + j < lv.w && gy < lv.h) {
                                out[l][(size_t)gy * lv.w + gx + j] = (word >> (8 * j)) & 255;
                                cnt[l][(size_t)gy * lv.w + gx + j]++;
                            }
                        }
                    }
                }
            }
            xoff += cw;
            yoff += ch;
            src_stride = dst_stride;
        }
    }
    long bad = 0, miss = 0;
    for (int l = 1; l < L; l++)
        for (size_t i = 0; i < out[l].size(); i++) {
            if (cnt[l][i] != 1) miss++;
            else if (out[l][i] != ref[lbase[l] + i]) bad++;
        }
    printf("%5dx%-5d L=%d tile %3dx%-2d items %5zu lds %6d tab %4d: %s (miss %ld, bad %ld)\n", W, H, L, tw, th,
           b.h_twr_items.size(), b.twr_lds, b.twr_tab_cap, (miss || bad) ? "MISMATCH" : "ok", miss, bad);
    if (miss || bad) fails++;
}

int main() {
    int sizes[][2] = {{1241, 376}, {1920, 1080}, {752, 480}, {97, 61}, {130, 77}, {33, 33}, {640, 17}, {257, 193},
                      {8192, 160}, {160, 8192}, {1, 1}, {2, 3}, {17, 9}, {400, 256}, {333, 201}, {1024, 768}};
    for (auto &s : sizes) run(s[0], s[1], TWR_TW, TWR_TH, 8, 1);
    for (auto &s : sizes) run(s[0], s[1], TWR_TW, TWR_TH, 12, 2);
    for (auto &s : sizes) run(s[0], s[1], TWR_TW, TWR_TH, 2, 6);
    for (auto &s : sizes) run(s[0], s[1], 64, 16, 3, 7);
    int tiles[][2] = {{16, 4}, {64, 16}, {128, 32}, {240, 64}, {200, 40}, {48, 8}, {240, 4}, {16, 64}};
    for (auto &t : tiles) {
        run(1241, 376, t[0], t[1], 8, 3);
        run(97, 61, t[0], t[1], 8, 4);
        run(1920, 1080, t[0], t[1], 8, 5);
    }
    printf("fails: %d\n", fails);
    return fails ? 1 : 0;
}
