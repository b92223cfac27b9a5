"""Pins of the oracle's smoothing, orientation, rBRIEF and stereo matcher.

Checks: scipy correlation with the same integer taps, trigonometric
identities of the Q14 tables, float atan2 away from bin boundaries, exact
180-degree rotation invariance, constant patches, a numpy brute-force
matcher and a pure translation whose disparity is known.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from synth import scenes
from synth.configs import Params

TAPS = np.array([18, 33, 49, 56, 49, 33, 18], dtype=np.int64)


def test_blur_matches_scipy_correlate():
    img = scenes.mono_image(3, 90, 70, 20)
    h = ndimage.correlate1d(img.astype(np.int64), TAPS, axis=1, mode="nearest")
    h = (h + 128) >> 8
    v = ndimage.correlate1d(h, TAPS, axis=0, mode="nearest")
    v = (v + 128) >> 8
    assert np.array_equal(oracle.blur_level(img), v.astype(np.uint8))
    assert TAPS.sum() == 256


def test_tables_identities():
    C, S = oracle.rot_table()
    bx, by = oracle.bin_table()
    for k in range(30):
        assert abs(C[k] ** 2 + S[k] ** 2 - 16384 ** 2) <= 2 * 16384
        assert C[(k + 15) % 30] == -C[k] and S[(k + 15) % 30] == -S[k]
        assert bx[(k + 15) % 30] == -bx[k] and by[(k + 15) % 30] == -by[k]
    assert (C[0], S[0]) == (16384, 0)
    assert (C[5], S[5]) == (8192, 14189)          # cos 60 deg is exactly 1/2
    assert (bx[7], by[7]) == (0, 16384)           # the 90-degree boundary


def test_angle_bin_vs_atan2():
    rng = np.random.default_rng(0)
    n_checked = 0
    for _ in range(4000):
        mx, my = rng.integers(-3_000_000, 3_000_000, 2)
        ang = np.degrees(np.arctan2(my, mx)) % 360.0
        frac = (ang - 6.0) / 12.0
        if abs(frac - np.round(frac)) < 1e-3:
            continue                               # too close to a boundary for float
        assert oracle.angle_bin(mx, my) == int(np.floor(ang / 12.0 + 0.5)) % 30
        n_checked += 1
    assert n_checked > 3900
    assert oracle.angle_bin(0, 0) == 0
    assert oracle.angle_bin(5, 0) == 0
    # 90 degrees lies exactly on the boundary at 6 + 12 * 7: it joins the upper bin
    assert oracle.angle_bin(0, 5) == 8


def _ramp_patch(phi_deg, size=41, a=128.0, b=3.0):
    c = size // 2
    v, u = np.mgrid[-c:c + 1, -c:c + 1]
    t = np.radians(phi_deg)
    return np.clip(np.rint(a + b * (u * np.cos(t) + v * np.sin(t))), 0, 255).astype(np.uint8)


def test_orientation_of_ramps():
    """The intensity centroid of a linear ramp points along its gradient, so
    the bin is the nearest multiple of 12 degrees (away from boundaries)."""
    for phi in np.arange(0.0, 360.0, 2.5):
        frac = (phi - 6.0) / 12.0
        if abs(frac - np.round(frac)) < 0.15:
            continue
        img = _ramp_patch(phi)
        m10, m01 = oracle.moments(img, 20, 20)
        assert oracle.angle_bin(m10, m01) == int(np.floor(phi / 12.0 + 0.5)) % 30, phi


def test_rotation_point_identities():
    for u in range(-15, 16):
        for v in range(-15, 16):
            if u * u + v * v > 225:
                continue
            assert oracle.rotate_point(u, v, 0) == (u, v)
            assert oracle.rotate_point(u, v, 15) == (-u, -v)
            for k in range(30):
                a = oracle.rotate_point(u, v, k)
                b = oracle.rotate_point(u, v, (k + 15) % 30)
                assert b == (-a[0], -a[1])
                assert abs(a[0]) <= 15 and abs(a[1]) <= 15


def _describe_one(img, x, y, pattern, blur=1):
    H, W = img.shape
    p = Params(n_levels=1, border=16, blur=blur)
    packed = img.reshape(-1).copy()
    kps = {k: np.zeros(1, t) for k, t in oracle.KP_FIELDS}
    kps["x"][0], kps["y"][0] = x, y
    return oracle.describe(packed, W, H, p, pattern, kps)


def test_constant_patch_descriptor_is_zero(pattern):
    img = np.full((64, 64), 77, np.uint8)
    d = _describe_one(img, 32, 32, pattern)
    assert d["bin"][0] == 0 and not d["desc"].any()


@pytest.mark.parametrize("seed", range(5))
def test_descriptor_rot180_invariance(seed, pattern):
    """Rotating the image by 180 degrees about the keypoint adds 15 to the
    bin and leaves the descriptor unchanged (odd rounding, symmetric blur)."""
    img = scenes.mono_image(seed, 81, 81, 15)
    a = _describe_one(img, 40, 40, pattern)
    b = _describe_one(img[::-1, ::-1].copy(), 40, 40, pattern)
    m = oracle.moments(img, 40, 40)
    if m != (0, 0):
        assert b["bin"][0] == (a["bin"][0] + 15) % 30
    assert np.array_equal(a["desc"], b["desc"])
    assert a["desc"].any()


def test_descriptor_bin0_direct(pattern):
    """With the keypoint oriented at bin 0 the tests use the pattern as is."""
    img = _ramp_patch(0.0, 81, 128.0, 1.0)
    img = img ^ (np.indices(img.shape).sum(0) % 3 == 0).astype(np.uint8)   # texture
    d = _describe_one(img, 40, 40, pattern, blur=0)
    assert d["bin"][0] == 0
    bits = [int(img[40 + pv, 40 + pu] < img[40 + qv, 40 + qu]) for pu, pv, qu, qv in pattern.astype(int)]
    words = [sum(bits[32 * w + i] << i for i in range(32)) for w in range(8)]
    assert list(d["desc"][0]) == words


def _brute_stereo(kl, kr, p):
    nl = len(kl["x"])
    idx = np.full(nl, -1, np.int64)
    dist = np.full(nl, 0xFFFF, np.int64)
    disp = np.full(nl, -1, np.int64)
    if len(kr["x"]) == 0:
        return idx, dist, disp
    bl = np.unpackbits(kl["desc"].view(np.uint8), axis=1)
    br = np.unpackbits(kr["desc"].view(np.uint8), axis=1)
    ham = (bl[:, None, :] != br[None, :, :]).sum(-1)
    for i in range(nl):
        dy = np.abs(kr["y"].astype(int) - int(kl["y"][i]))
        d = int(kl["x0"][i]) - kr["x0"].astype(int)
        ok = (kr["level"] == kl["level"][i]) & (dy <= p.row_band) & (d >= 0) & (d <= p.d_max)
        js = np.nonzero(ok)[0]
        if len(js) == 0:
            continue
        order = np.lexsort((js, d[js], dy[js], ham[i, js]))
        j = js[order[0]]
        if ham[i, j] <= p.match_th:
            idx[i], dist[i], disp[i] = j, ham[i, j], d[j]
    return idx, dist, disp


def test_stereo_vs_bruteforce(pattern):
    p = Params()
    left, right = scenes.stereo_pair(21, 320, 200, 60, 40)
    kl, kr, (idx, dist, disp) = oracle.frontend_pair(left, right, p, pattern)
    bi, bd, bp = _brute_stereo(kl, kr, p)
    assert (idx >= 0).sum() > 20
    assert np.array_equal(idx, bi) and np.array_equal(dist, bd) and np.array_equal(disp, bp)


def test_stereo_pure_translation(pattern):
    """Right view = left shifted by d px: level-0 matches recover d."""
    d = 13
    base = scenes.mono_image(8, 360, 160, 70)
    left = base[:, :320].copy()
    right = base[:, d:320 + d].copy()
    p = Params(n_levels=1)
    kl, kr, (idx, dist, disp) = oracle.frontend_pair(left, right, p, pattern)
    # the cell grids of the two views are offset by d, so only keypoints whose
    # translated twin was also culled have a known answer: that twin, at distance 0
    right_at = {(int(x), int(y)): j for j, (x, y) in enumerate(zip(kr["x"], kr["y"]))}
    n_twin = 0
    for i in range(len(kl["x"])):
        j = right_at.get((int(kl["x"][i]) - d, int(kl["y"][i])))
        if j is None:
            continue
        n_twin += 1
        assert (idx[i], dist[i], disp[i]) == (j, 0, d)
    assert n_twin > 15
