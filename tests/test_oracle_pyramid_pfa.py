"""Pins of the oracle's pyramid, projection, PFA and keypoint cap.

Checks: the paper's cell-size statement and PFA worked example (fixtures in
tests/golden), float evaluations of the level-size and projection rules,
scipy bilinear resampling within its rounding bound, constant images, a
brute-force sparse PFA on random records, and invariants on real scenes.
"""
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import scenes
from synth.configs import Params

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_cell_sizes_paper_statement():
    with open(os.path.join(GOLDEN, "cell_sizes.txt")) as f:
        line = [l for l in f if l.startswith("level7_cell")][0]
    assert oracle.cell_size(32, 7) == int(line.split(":")[1])
    # cells shrink with the level scale and never below floor(32 / 1.2^l)
    for l in range(8):
        assert oracle.cell_size(32, l) == int(np.floor(32 / 1.2 ** l + 1e-9))


@pytest.mark.parametrize("W,H", [(1241, 376), (752, 480), (1920, 1080), (640, 480), (97, 61)])
def test_level_sizes_float(W, H):
    for l in range(8):
        w, h = oracle.level_size(W, H, l)
        assert (w, h) == (int(np.floor(W / 1.2 ** l + 0.5)), int(np.floor(H / 1.2 ** l + 0.5)))


def test_scale_and_projection():
    for l in range(8):
        assert oracle.scale_q16(l) == int(round(65536 * 1.2 ** l))
    # within half a pixel of x * 1.2^l (plus the Q16 rounding of the factor)
    for l in range(8):
        for x in range(0, 1700, 37):
            x0 = oracle.project(x, l, 10 ** 6)
            assert abs(x0 - x * 1.2 ** l) <= 0.5 + x * 1e-5
    # projections of distinct pixels of one level never collide (spacing >= 1.2)
    for l in range(1, 8):
        xs = [oracle.project(x, l, 10 ** 6) for x in range(2000)]
        assert len(set(xs)) == len(xs)
    assert oracle.project(5000, 0, 100) == 99      # clamp to the image


def test_pyramid_constant():
    img = np.full((376, 1241), 137, dtype=np.uint8)
    for lvl in oracle.pyramid(img, 8):
        assert lvl.min() == lvl.max() == 137


def test_pyramid_vs_float_bilinear():
    """Each level equals the float bilinear resample (half-pixel centres,
    clamp-to-edge) of the previous level to within 1 grey level."""
    img = scenes.mono_image(5, 300, 200, 40)
    levels = oracle.pyramid(img, 6)
    for l in range(1, 6):
        src, dst = levels[l - 1].astype(np.float64), levels[l]
        h, w = dst.shape
        sh, sw = src.shape
        ys = (np.arange(h) + 0.5) * sh / h - 0.5
        xs = (np.arange(w) + 0.5) * sw / w - 0.5
        gy, gx = np.meshgrid(ys, xs, indexing="ij")
        ref = ndimage.map_coordinates(src, [gy, gx], order=1, mode="nearest")
        diff = np.abs(ref - dst.astype(np.float64))
        # Q8 flooring moves each source coordinate by < 1/256 px, i.e. by at
        # most 255/256 grey levels per axis, plus 1/2 for the final rounding
        assert diff.max() < 0.5 + 2 * 255.0 / 256.0
        assert np.mean(diff) < 0.6


def _q8_positions(n_dst, n_src):
    """Half-pixel-centre source coordinate of every output index,
    (o + 1/2) n_src / n_dst - 1/2, floored to a multiple of 1/256."""
    from fractions import Fraction
    out = []
    for o in range(n_dst):
        u = (Fraction(2 * o + 1) * n_src / n_dst - 1) / 2
        out.append(float(Fraction(int(np.floor(u * 256)), 256)))
    return np.array(out)


@pytest.mark.parametrize("seed,W,H", [(1, 61, 47), (2, 300, 200), (3, 97, 256), (4, 1241, 40)])
def test_pyramid_level_is_rounded_bilinear_exactly(seed, W, H):
    """Each level, taken from the oracle's previous level, equals scipy's
    bilinear value at the Q8-floored half-pixel-centre coordinate rounded
    half up, exactly.  Every product of a Q8 weight and a byte is exact in
    float64, so scipy's value is the exact rational one; exact halves occur
    (asserted), so a round-half-down or a truncating slip fails here."""
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, (H, W)).astype(np.uint8)
    levels = oracle.pyramid(img, 6)
    ties = 0
    for l in range(1, 6):
        src, dst = levels[l - 1].astype(np.float64), levels[l]
        h, w = dst.shape
        sh, sw = src.shape
        gy, gx = np.meshgrid(_q8_positions(h, sh), _q8_positions(w, sw), indexing="ij")
        v = ndimage.map_coordinates(src, [gy, gx], order=1, mode="nearest", prefilter=False)
        ref = np.floor(v + 0.5)
        assert np.array_equal(ref, dst.astype(np.float64)), (l, np.argwhere(ref != dst)[:3])
        ties += int(np.sum(v - np.floor(v) == 0.5))
    assert ties > 0


def test_pyramid_ramp_exact_to_one():
    """A linear ramp is resampled to the ramp at the mapped coordinate."""
    x = np.arange(256, dtype=np.float64)
    img = np.tile(np.clip(np.round(x * 0.8 + 10), 0, 255).astype(np.uint8), (40, 1))
    lv = oracle.pyramid(img, 3)
    w1 = lv[1].shape[1]
    xs = (np.arange(w1) + 0.5) * 256 / w1 - 0.5
    ref = np.clip(xs, 0, 255) * 0.8 + 10
    assert np.abs(lv[1][20].astype(np.float64) - ref)[1:-1].max() <= 1.0


def _load_pfa_figure():
    recs, K, keep, sup = [], {}, set(), set()
    with open(os.path.join(GOLDEN, "pfa_figure.txt")) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "K":
                K[(int(t[1]), int(t[2]))] = (int(t[3]), int(t[4]))
            elif t[0] == "KEEP":
                keep.add((int(t[1]), int(t[2])))
            elif t[0] == "SUPPRESS":
                sup.add((int(t[1]), int(t[2])))
            else:
                recs.append(tuple(int(v) for v in t))
    return recs, K, keep, sup


@pytest.mark.parametrize("mode", [0, 1])
def test_pfa_paper_figure(mode):
    recs, K, keep, sup = _load_pfa_figure()
    level = [r[0] for r in recs]
    y0 = [r[1] for r in recs]
    x0 = [r[2] for r in recs]
    resp = [r[3] for r in recs]
    kl, kr, kp = oracle.pfa_from_records(level, x0, y0, resp, 5, 5, 3, nms_mode=mode)
    for i, r in enumerate(recs):
        pos = (r[1], r[2])
        assert (kl[i], kr[i]) == K[pos]
        assert kp[i] == (pos in keep)
        assert (not kp[i]) == (pos in sup)
    # survivors are re-emitted at every level they were detected on
    assert sum(1 for i, r in enumerate(recs) if kp[i] and (r[1], r[2]) == (1, 1)) == 3


def _brute_pfa(level, x0, y0, resp, mode, radius=1):
    """Sparse O(n^2) definition: group by native position, compare windows."""
    n = len(level)
    kl = np.zeros(n, int)
    kr = np.zeros(n, int)
    for i in range(n):
        same = [j for j in range(n) if x0[j] == x0[i] and y0[j] == y0[i]]
        kl[i] = len(same)
        kr[i] = sum(resp[j] for j in same)
    keep = np.ones(n, bool)
    for i in range(n):
        for j in range(n):
            if (x0[j], y0[j]) == (x0[i], y0[i]):
                continue
            if abs(x0[j] - x0[i]) <= radius and abs(y0[j] - y0[i]) <= radius:
                if mode == 0:
                    b = kl[j] > kl[i] or (kl[j] == kl[i] and kr[j] > kr[i])
                else:
                    b = kl[j] > kl[i] and kr[j] > kr[i]
                if b:
                    keep[i] = False
    return kl, kr, keep


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mode", [0, 1])
def test_pfa_vs_bruteforce(seed, mode):
    rng = np.random.default_rng(seed)
    n_lv, W, H = 4, 14, 12
    level, x0, y0, resp = [], [], [], []
    for l in range(n_lv):
        # distinct positions per level (one keypoint per level per pixel)
        cells = rng.choice(W * H, size=rng.integers(5, 20), replace=False)
        for c in cells:
            level.append(l)
            x0.append(int(c % W))
            y0.append(int(c // W))
            resp.append(int(rng.integers(1, 6)) * 10)
    kl, kr, keep = oracle.pfa_from_records(level, x0, y0, resp, W, H, n_lv, nms_mode=mode)
    bkl, bkr, bkeep = _brute_pfa(level, x0, y0, resp, mode)
    assert np.array_equal(kl, bkl) and np.array_equal(kr, bkr)
    assert np.array_equal(keep, bkeep)


def test_detect_invariants_and_cap():
    img = scenes.mono_image(11, 400, 300, 80)
    p = Params(n_max=100000, border=16)
    packed = oracle.pyramid_packed(img, p.n_levels)
    full = oracle.detect(packed, 400, 300, p)
    nopfa = oracle.detect(packed, 400, 300, Params(n_max=100000, border=16, pfa=0))
    assert len(full["x"]) > 50
    # survivors are a subset of the culled keypoints; k_l bounded by the levels
    culled = set(zip(nopfa["level"], nopfa["x"], nopfa["y"]))
    assert set(zip(full["level"], full["x"], full["y"])) <= culled
    assert full["kl"].max() <= p.n_levels and full["kl"].min() >= 1
    assert len(full["x"]) < len(nopfa["x"])            # PFA lowers the count (Sec. IV-B-2)
    # canonical order
    order = np.lexsort((full["x"], full["y"], full["level"]))
    lv_c = [oracle.cell_size(p.cell0, l) for l in full["level"]]
    cy = full["y"] // np.array(lv_c)
    key = full["level"].astype(np.int64) * 10 ** 8 + cy * 10 ** 4 + full["x"] // np.array(lv_c)
    assert np.all(np.diff(key) > 0)
    # cap: the first n_max by (k_l desc, k_r desc, canonical asc)
    n_max = 40
    capped = oracle.detect(packed, 400, 300, Params(n_max=n_max, border=16))
    assert len(capped["x"]) == n_max
    rank = np.lexsort((np.arange(len(key)), -full["kr"].astype(np.int64), -full["kl"].astype(np.int64)))
    chosen = set(np.sort(rank[:n_max]))
    got = set(zip(capped["level"], capped["x"], capped["y"]))
    exp = set((full["level"][i], full["x"][i], full["y"][i]) for i in chosen)
    assert got == exp


def test_gated_detect_subset():
    img = scenes.mono_image(12, 320, 256, 60)
    p = Params(border=16)
    packed = oracle.pyramid_packed(img, p.n_levels)
    full = oracle.detect(packed, 320, 256, p)
    ones = np.ones((8, 10), np.uint8)
    same = oracle.detect(packed, 320, 256, p, ones)
    assert all(np.array_equal(full[k], same[k]) for k in ("x", "y", "level", "kr"))
    none = oracle.detect(packed, 320, 256, p, np.zeros((8, 10), np.uint8))
    assert len(none["x"]) == 0
