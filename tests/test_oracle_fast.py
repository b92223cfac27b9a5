"""Pins of the oracle's FAST + Bounded Rectification and Feature Culling.

Each test checks the oracle against something other than itself: closed-form
counts, the paper's worked non-corner example, hand-built patches whose
labels follow from Eq. 1-3, a geometric theorem (a straight step edge is
never a corner), exact symmetries, and a numpy argmax over cells.
"""
import numpy as np
import pytest

import oracle
from synth import scenes

# ring offsets (dx, dy) of the radius-3 Bresenham circle, cyclic order as
# drawn in the paper's non-corner figure (Sec. II-A)
RING = [(0, -3), (1, -3), (2, -2), (3, -1), (3, 0), (3, 1), (2, 2), (1, 3),
        (0, 3), (-1, 3), (-2, 2), (-3, 1), (-3, 0), (-3, -1), (-2, -2), (-1, -3)]


def test_lut_counts_closed_form():
    """A mask whose longest cyclic run is exactly r (9 <= r <= 14) is a run of
    r ones bounded by two zeros (16 placements) with 14 - r free bits; r = 15
    has 16 masks and r = 16 one.  BR accepts r in [9, 13]; plain FAST r >= 9."""
    br = sum(16 * 2 ** (14 - r) for r in range(9, 14))
    plain = br + 16 * 2 ** 0 + 16 + 1
    assert (br, plain) == (992, 1025)
    got_br = sum(oracle.mask_is_corner(m, 9, 13) for m in range(1 << 16))
    got_plain = sum(oracle.mask_is_corner(m, 9, 16) for m in range(1 << 16))
    assert (got_br, got_plain) == (992, 1025)


def test_longest_run_special_cases():
    assert oracle.longest_run([0] * 16) == 0
    assert oracle.longest_run([1] * 16) == 16
    wrap = [1] * 5 + [0] * 6 + [1] * 5          # run wraps through index 0
    assert oracle.longest_run(wrap) == 10
    alt = [1, 0] * 8
    assert oracle.longest_run(alt) == 1


def test_cardinal_prefilter_property():
    """Any cyclic run of >= 9 covers two consecutive compass points (0, 4, 8,
    12); a GPU prefilter relies on it."""
    for m in range(1 << 16):
        if oracle.mask_is_corner(m, 9, 16):
            c = [(m >> k) & 1 for k in (0, 4, 8, 12)]
            assert any(c[i] and c[(i + 1) % 4] for i in range(4)), hex(m)


def _patch(center, ring_vals, size=7):
    p = np.full((size, size), center, dtype=np.uint8)
    c = size // 2
    for (dx, dy), v in zip(RING, ring_vals):
        p[c + dy, c + dx] = v
    return p


def test_paper_noncorner_example():
    """Fig. "noncorner": all 16 ring pixels bright.  Plain FAST (Eq. 2) calls
    it a corner; Bounded Rectification (Eq. 3, P_max = 13) rejects it."""
    p = _patch(100, [200] * 16)
    br, nb, nd = oracle.is_corner(p, 3, 3, 20, 9, 13)
    plain, _, _ = oracle.is_corner(p, 3, 3, 20, 9, 16)
    assert nb == 16 and nd == 0
    assert plain and not br


def test_label_equality_is_similar():
    """|I_p - I_c| = eps is neither bright nor dark."""
    ring = [120] * 9 + [100] * 7
    p = _patch(100, ring)
    assert not oracle.is_corner(p, 3, 3, 20)[0]
    ring = [121] * 9 + [100] * 7
    p = _patch(100, ring)
    ok, nb, nd = oracle.is_corner(p, 3, 3, 20)
    assert ok and nb == 9
    ring = [79] * 10 + [100] * 6
    ok, nb, nd = oracle.is_corner(_patch(100, ring), 3, 3, 20)
    assert ok and nd == 10
    ring = [80] * 10 + [100] * 6
    assert not oracle.is_corner(_patch(100, ring), 3, 3, 20)[0]


def test_run_length_bounds():
    for r in range(0, 17):
        ring = [200] * r + [100] * (16 - r)
        ok, nb, _ = oracle.is_corner(_patch(100, ring), 3, 3, 20, 9, 13)
        assert nb == r
        assert ok == (9 <= r <= 13)


def test_flat_and_isolated_pixel():
    img = np.full((24, 24), 90, dtype=np.uint8)
    assert oracle.crf(img, 20, 9, 13, 3).max() == 0
    img[12, 12] = 250
    assert oracle.crf(img, 20, 9, 13, 3)[12, 12] == 0      # N_d = 16 -> rejected by BR
    assert oracle.crf(img, 20, 9, 16, 3)[12, 12] == 16 * 160


def test_square_corner_is_br_corner():
    """The corner pixel of a bright quadrant: 5 ring pixels inside, the other
    11 contiguous ones dark -> N_d = 11 and a BR corner."""
    img = np.full((24, 24), 40, dtype=np.uint8)
    img[10:, 10:] = 200
    ok, nb, nd = oracle.is_corner(img, 10, 10, 20)
    assert ok and nd == 11 and nb == 0
    assert oracle.score(img, 10, 10) == 11 * 160


def test_step_edge_never_corner():
    """A straight two-level edge puts at most 8 contiguous ring pixels on the
    side opposite the centre, so no pixel passes even plain FAST-9."""
    rng = np.random.default_rng(3)
    yy, xx = np.mgrid[0:40, 0:40] + 0.5
    for _ in range(60):
        th = rng.uniform(0, 2 * np.pi)
        off = rng.uniform(-5, 5)
        inside = (xx - 20) * np.cos(th) + (yy - 20) * np.sin(th) > off
        img = np.where(inside, 210, 30).astype(np.uint8)
        assert oracle.crf(img, 20, 9, 16, 3).max() == 0


def _scene_crop(seed, w=96, h=80):
    return scenes.mono_image(seed, w, h, n_polygons=25)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_crf_symmetries(seed):
    """The ring is symmetric under 180-degree rotation and transposition and
    the response is |.|-symmetric, so CRF commutes with these maps and is
    invariant to 255 - I."""
    for img in (_scene_crop(seed), scenes.random_image(seed, 40, 36)):
        base = oracle.crf(img, 20, 9, 13, 3)
        assert base.max() > 0
        assert np.array_equal(oracle.crf(img[::-1, ::-1].copy(), 20, 9, 13, 3), base[::-1, ::-1])
        assert np.array_equal(oracle.crf(img.T.copy(), 20, 9, 13, 3), base.T)
        assert np.array_equal(oracle.crf((255 - img).astype(np.uint8), 20, 9, 13, 3), base)


def _cell_argmax(crf_map, c, border):
    """numpy reference of the per-cell max key over a given response map."""
    H, W = crf_map.shape
    ncx, ncy = (W + c - 1) // c, (H + c - 1) // c
    out = np.zeros((ncy, ncx), dtype=np.uint32)
    for cy in range(ncy):
        for cx in range(ncx):
            blk = crf_map[cy * c:(cy + 1) * c, cx * c:(cx + 1) * c].astype(np.int64)
            if blk.max() == 0:
                continue
            ys, xs = np.nonzero(blk == blk.max())
            first = np.lexsort((xs, ys))[0]
            idx = ys[first] * c + xs[first]
            out[cy, cx] = (int(blk.max()) << 10) | (1023 - idx)
    return out


@pytest.mark.parametrize("c", [32, 13, 8])
def test_cull_matches_cell_argmax(c):
    from synth.configs import Params
    img = _scene_crop(7, 120, 90)
    p = Params(eps_hi=20, eps_lo=-1, border=3)
    key, flag = oracle.cull_level(img, c, p)
    ref = _cell_argmax(oracle.crf(img, 20, 9, 13, 3), c, 3)
    assert np.array_equal(key, ref)
    assert flag.sum() == 0


def test_cull_tie_goes_to_first_raster_pixel():
    from synth.configs import Params
    img = np.full((40, 40), 40, dtype=np.uint8)
    img[10:14, 10:14] = 200          # two identical squares in one 32-px cell
    img[20:24, 20:24] = 200
    key, _ = oracle.cull_level(img, 32, Params(eps_hi=20, eps_lo=-1, border=3))
    idx = 1023 - (int(key[0, 0]) & 1023)
    y, x = idx // 32, idx % 32
    assert 10 <= y < 14 and 10 <= x < 14                  # inside the first square
    crf = oracle.crf(img, 20, 9, 13, 3)
    assert crf[y, x] == crf[y + 10, x + 10] == int(key[0, 0]) >> 10   # tied with its twin


def test_fallback_threshold():
    from synth.configs import Params
    img = np.full((40, 40), 100, dtype=np.uint8)
    img[12:, 12:] = 112              # contrast 12: only the eps_lo = 7 test fires
    key, flag = oracle.cull_level(img, 32, Params(eps_hi=20, eps_lo=7, border=3))
    assert key[0, 0] != 0 and flag[0, 0] == 1
    key2, flag2 = oracle.cull_level(img, 32, Params(eps_hi=20, eps_lo=-1, border=3))
    assert key2[0, 0] == 0
    img[30:, 30:] = 160              # a strong corner elsewhere in the cell wins outright
    key3, flag3 = oracle.cull_level(img, 32, Params(eps_hi=20, eps_lo=7, border=3))
    assert flag3[0, 0] == 0 and key3[0, 0] != 0
