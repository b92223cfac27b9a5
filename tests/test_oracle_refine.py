"""Pins of the sub-pixel stereo refinement oracle (``or_stereo_refine``).

The refinement minimises the SAD of a (2w+1)^2 window over shifts of the
matched right column and fits a parabola through the three SADs around the
minimum.  The pins come from closed forms, not from the oracle's code:

* an intensity ramp shifted by d + t gives SAD(s) = (2w+1)^2 |c (s + t)|
  (a V), whose three-point parabola has its vertex at -t / (1 - t) / 2
  pixels from the integer minimum for t in (0, 1/2]: exactly the half
  pixel for t = 1/2, the known bias of parabola fitting on a V otherwise;
* a textured patch copied at an integer shift has SAD 0 at that shift;
* a flat patch has equal SADs, so the least |s| wins and the offset is 0;
* a minimum at the end of the search range, a missing match and a window
  that leaves the level are not refined;
* a level-l keypoint scales its level disparity by S_l = round(65536 1.2^l).
"""
import numpy as np
import pytest

import oracle

INT32_MIN = -(2 ** 31)


def kp_dicts(xl, yl, xr, level):
    n = len(xl)

    def one(x, y):
        d = {k: np.zeros(n, dtype=t) for k, t in oracle.KP_FIELDS}
        d["x"][:] = x
        d["y"][:] = y
        d["level"][:] = level
        return d

    return one(xl, yl), one(xr, yl)


def packed_single_level(img_l, img_r, W, H, level):
    """Packed pyramids whose level `level` holds the given images (other
    levels zero): the refinement reads only the keypoints' level."""
    sizes = [oracle.level_size(W, H, l) for l in range(level + 1)]
    assert sizes[level] == (img_l.shape[1], img_l.shape[0])
    total = sum(w * h for w, h in sizes)
    out = []
    for img in (img_l, img_r):
        buf = np.zeros(total, np.uint8)
        at = sum(w * h for w, h in sizes[:level])
        buf[at:at + img.size] = img.reshape(-1)
        out.append(buf)
    return out


def rhaz(v):
    """round half away from zero of a float that is a multiple of 1/8 or a
    ratio away from ties (exact here)"""
    return int(np.sign(v) * np.floor(abs(v) + 0.5))


@pytest.mark.parametrize("t8", [1, 2, 3, 4])
@pytest.mark.parametrize("d", [0, 3, 17])
def test_ramp_fractional_shift_closed_form(t8, d):
    # L(x) = 8 (x - c0) + 64, R(x) = L(x + d + t) with t = t8 / 8: exact bytes
    # over every window the refinement reads (c0 = xl - 5)
    W, H = 100, 40
    xl = d + 15                                         # the right search starts at column 5
    c0 = xl - 5
    x = np.arange(W)
    L = np.tile((8 * (x - c0) + 64) % 256, (H, 1)).astype(np.uint8)
    R = np.tile((8 * (x + d - c0) + t8 + 64) % 256, (H, 1)).astype(np.uint8)
    pl, pr = packed_single_level(L, R, W, H, 0)
    kl, kr = kp_dicts(np.array([xl] * 3), [12, 20, 28], np.array([xl - d] * 3), 0)
    disp, sad = oracle.stereo_refine(pl, pr, W, H, kl, kr, np.arange(3), 5, 5)
    t = t8 / 8.0
    # SAD(s) = 121 * 8 |s + t|: minimum at s = 0, parabola vertex at
    # -t / (1 - t) / 2 pixels, so the disparity grows by t / (1 - t) / 2
    exp = 256 * d + rhaz(128.0 * t / (1.0 - t))
    assert list(disp) == [exp] * 3, (disp, exp)
    assert list(sad) == [121 * t8] * 3
    if t8 == 4:
        assert exp == 256 * d + 128                    # the half pixel exactly


def test_textured_integer_shift():
    rng = np.random.default_rng(5)
    W, H = 120, 50
    L = rng.integers(0, 256, (H, W)).astype(np.uint8)
    d = 9
    R = np.zeros_like(L)
    R[:, :W - d] = L[:, d:]                             # R(x) = L(x + d)
    xl = np.array([40, 55, 70, 85])
    err = np.array([-4, -1, 2, 4])                      # wrong integer guesses within the range
    pl, pr = packed_single_level(L, R, W, H, 0)
    kl, kr = kp_dicts(xl, [25] * 4, xl - d + err, 0)
    disp, sad = oracle.stereo_refine(pl, pr, W, H, kl, kr, np.arange(4), 5, 5)
    assert list(sad) == [0] * 4
    # integer part: the true disparity; the sub-pixel part stays within 1/2
    assert np.all(np.abs(disp - 256 * d) <= 128)


def test_flat_patch_and_not_refined_cases():
    W, H = 80, 40
    flat = np.full((H, W), 77, np.uint8)
    pl, pr = packed_single_level(flat, flat, W, H, 0)
    kl, kr = kp_dicts(np.array([30]), [20], np.array([26]), 0)
    disp, sad = oracle.stereo_refine(pl, pr, W, H, kl, kr, np.array([0]), 5, 5)
    assert disp[0] == 256 * 4 and sad[0] == 0          # offset 0, shift 0
    # no match
    disp, sad = oracle.stereo_refine(pl, pr, W, H, kl, kr, np.array([-1]), 5, 5)
    assert disp[0] == INT32_MIN and sad[0] == 0xFFFFFFFF
    # windows leaving the level (left at the border, right search at the edge)
    kl2, kr2 = kp_dicts(np.array([3, 30]), [20, 20], np.array([26, 72]), 0)
    disp, _ = oracle.stereo_refine(pl, pr, W, H, kl2, kr2, np.array([0, 1]), 5, 5)
    assert list(disp) == [INT32_MIN, INT32_MIN]
    # minimum at the end of the search range: a ramp guess off by 7 > r
    x = np.arange(W)
    L = np.tile(3 * x, (H, 1)).astype(np.uint8)
    pl, pr = packed_single_level(L, L, W, H, 0)
    kl3, kr3 = kp_dicts(np.array([40]), [20], np.array([47]), 0)
    disp, _ = oracle.stereo_refine(pl, pr, W, H, kl3, kr3, np.array([0]), 5, 5)
    assert disp[0] == INT32_MIN
    # within the range it refines to the exact integer shift
    kl4, kr4 = kp_dicts(np.array([40]), [20], np.array([44]), 0)
    disp, sad = oracle.stereo_refine(pl, pr, W, H, kl4, kr4, np.array([0]), 5, 5)
    assert disp[0] == 0 and sad[0] == 0


@pytest.mark.parametrize("level", [1, 2, 5])
def test_level_scaling(level):
    W0, H0 = 400, 240
    w, h = oracle.level_size(W0, H0, level)
    x = np.arange(w)
    d = 6
    xl = d + 15
    c0 = xl - 5
    L = np.tile((8 * (x - c0) + 64) % 256, (h, 1))
    R = np.tile((8 * (x + d - c0) + 4 + 64) % 256, (h, 1))   # level shift d + 1/2
    pl, pr = packed_single_level(L.astype(np.uint8), R.astype(np.uint8), W0, H0, level)
    kl, kr = kp_dicts(np.array([xl]), [h // 2], np.array([xl - d]), level)
    disp, _ = oracle.stereo_refine(pl, pr, W0, H0, kl, kr, np.array([0]), 5, 5)
    S = int(oracle.scale_q16(level))
    d_level = 256 * d + 128
    assert disp[0] == (d_level * S + 32768) // 65536
    assert abs(disp[0] / 256.0 - (d + 0.5) * 1.2 ** level) < 0.01


def test_window_and_radius_parameters():
    rng = np.random.default_rng(8)
    W, H = 90, 60
    L = rng.integers(0, 256, (H, W)).astype(np.uint8)
    R = np.zeros_like(L)
    R[:, :W - 5] = L[:, 5:]
    pl, pr = packed_single_level(L, R, W, H, 0)
    for w, r, err in ((1, 1, 1), (3, 2, -2), (7, 16, 11)):
        kl, kr = kp_dicts(np.array([45]), [30], np.array([40 + err]), 0)
        disp, sad = oracle.stereo_refine(pl, pr, W, H, kl, kr, np.array([0]), w, r)
        if abs(err) < r:
            assert sad[0] == 0 and abs(disp[0] - 256 * 5) <= 128, (w, r)
        else:
            assert disp[0] == INT32_MIN, (w, r)


def test_half_tie_rounds_away_from_zero():
    """Flat views with one bumped column on each side of the match give
    SAD(s < 0) = A, SAD(0) = 0, SAD(s > 0) = B: the vertex lies at
    (A - B) / (2 (A + B)) pixels.  A = 259, B = 253 put it at exactly
    1.5 / 256 pixel, which rounds away from zero to 2 / 256."""
    W, H = 80, 40
    L = np.full((H, W), 100, np.uint8)
    R = L.copy()
    xl, yl, xr = 40, 20, 36
    rows = slice(yl - 5, yl + 6)
    R[rows, xr - 6] = 100 + 23
    R[yl, xr - 6] = 100 + 29                         # column sum 10 * 23 + 29 = 259
    R[rows, xr + 6] = 100 + 23                       # column sum 253
    pl, pr = packed_single_level(L, R, W, H, 0)
    kl, kr = kp_dicts(np.array([xl]), [yl], np.array([xr]), 0)
    disp, sad = oracle.stereo_refine(pl, pr, W, H, kl, kr, np.array([0]), 5, 5)
    assert sad[0] == 0
    # refined right column 256 xr + 2 (the vertex moves toward the smaller side B)
    assert disp[0] == 256 * (xl - xr) - 2
    # mirrored: the offset changes sign, still rounded away from zero
    R2 = L.copy()
    R2[rows, xr + 6] = 100 + 23
    R2[yl, xr + 6] = 100 + 29
    R2[rows, xr - 6] = 100 + 23
    pl, pr = packed_single_level(L, R2, W, H, 0)
    disp, _ = oracle.stereo_refine(pl, pr, W, H, kl, kr, np.array([0]), 5, 5)
    assert disp[0] == 256 * (xl - xr) + 2


def test_equal_minima_either_side_take_the_negative_shift():
    """A period-2 texture copied with a one-column shift matches at s = -1
    and s = +1 equally (SAD 0) and not at s = 0: the tie goes to the
    smaller shift, -1."""
    W, H = 80, 40
    x = np.arange(W)
    L = np.tile(np.where(x % 2 == 0, 60, 180), (H, 1)).astype(np.uint8)
    R = np.tile(np.where(x % 2 == 1, 60, 180), (H, 1)).astype(np.uint8)   # R(x) = L(x + 1)
    xl, xr = 40, 30
    pl, pr = packed_single_level(L, R, W, H, 0)
    kl, kr = kp_dicts(np.array([xl]), [20], np.array([xr]), 0)
    disp, sad = oracle.stereo_refine(pl, pr, W, H, kl, kr, np.array([0]), 5, 5)
    assert sad[0] == 0
    # s* = -1, neighbours SAD(-2) = SAD(0): offset 0
    assert disp[0] == 256 * (xl - (xr - 1))
