"""Pins of the descriptor-matching oracle (``or_feature_match``): the frame
matched against itself, a known translation, the window and level-band
edges, the ratio test on constructed distances, the acceptance threshold
and invariance under a permutation of the references."""
import numpy as np
import pytest

import oracle
from synth import pattern as pat
from synth import scenes
from synth.configs import Params


@pytest.fixture(scope="module")
def frame():
    img = scenes.mono_image(31, 400, 300, 80)
    _, k = oracle.frontend_image(img, Params(), pat.brief_pattern())
    assert len(k["x"]) > 100
    return k


def flip_bits(desc, n, rng):
    """desc with n distinct random bits flipped (Hamming distance n)."""
    out = desc.copy()
    for b in rng.choice(256, n, replace=False):
        out[b >> 5] ^= np.uint32(1 << (b & 31))
    return out


def refs(x0, y0, level, desc):
    return {"x0": np.asarray(x0, np.uint16), "y0": np.asarray(y0, np.uint16),
            "level": np.asarray(level, np.uint8), "desc": np.asarray(desc, np.uint32).reshape(-1, 8)}


def test_self_match(frame):
    idx, d1, _ = oracle.feature_match(frame, frame, 0, 0, 256, 0)
    assert np.array_equal(idx, np.arange(len(idx)))
    assert np.all(d1 == 0)


def test_translation(frame):
    k = dict(frame)
    k["x0"] = frame["x0"].astype(np.int64) + 7
    k["y0"] = frame["y0"].astype(np.int64) + 5
    k = refs(k["x0"], k["y0"], frame["level"], frame["desc"])
    uniq = len({tuple(d) for d in frame["desc"]}) == len(frame["desc"])
    assert uniq
    idx, d1, _ = oracle.feature_match(frame, k, 7, 0, 256, 0)
    assert np.array_equal(idx, np.arange(len(idx))) and np.all(d1 == 0)
    # one pixel short in x: a keypoint's own moved copy is out of the window
    # (other keypoints' copies may still be candidates)
    idx, d1, _ = oracle.feature_match(frame, k, 6, 0, 256, 0)
    assert not np.any(idx == np.arange(len(idx)))
    assert np.all(d1 > 0)


def test_level_band():
    rng = np.random.default_rng(2)
    q = rng.integers(0, 2 ** 32, 8, dtype=np.uint64).astype(np.uint32)
    kq = refs([100], [50], [1], q)
    kr = refs([100], [50], [3], q)
    assert oracle.feature_match(kq, kr, 4, 1, 256, 0)[0][0] == -1
    assert oracle.feature_match(kq, kr, 4, 2, 256, 0)[0][0] == 0


def test_ratio_test_and_threshold():
    rng = np.random.default_rng(3)
    q = rng.integers(0, 2 ** 32, 8, dtype=np.uint64).astype(np.uint32)
    kq = refs([60], [60], [0], q)
    for d_best, d_second, ratio, accepted in ((10, 11, 90, False), (10, 12, 90, True), (10, 11, 0, True),
                                              (20, 20, 100, False), (0, 1, 90, True), (30, 40, 75, False)):
        descs = [flip_bits(q, d_second, rng), flip_bits(q, d_best, rng), flip_bits(q, 200, rng)]
        kr = refs([61, 59, 60], [60, 62, 58], [0, 0, 0], np.stack(descs))
        idx, d1, d2 = oracle.feature_match(kq, kr, 2, 0, 256, ratio)
        assert (d1[0], d2[0]) == (d_best, d_second)
        assert idx[0] == (1 if accepted else -1), (d_best, d_second, ratio)
    # equal distances: the smaller reference index wins when accepted
    descs = [flip_bits(q, 9, rng), flip_bits(q, 9, rng)]
    kr = refs([60, 60], [61, 59], [0, 0], np.stack(descs))
    idx, d1, d2 = oracle.feature_match(kq, kr, 1, 0, 256, 0)
    assert idx[0] == 0 and d1[0] == d2[0] == 9
    # a single candidate passes the ratio test; the threshold still applies
    kr = refs([60], [60], [0], flip_bits(q, 70, rng))
    idx, d1, d2 = oracle.feature_match(kq, kr, 0, 0, 64, 90)
    assert idx[0] == -1 and d1[0] == 70 and d2[0] == 0xFFFF
    idx, _, _ = oracle.feature_match(kq, kr, 0, 0, 70, 90)
    assert idx[0] == 0


def test_reference_permutation(frame):
    rng = np.random.default_rng(4)
    # references: the frame moved by up to 3 pixels with noisy descriptors
    n = len(frame["x0"])
    x0 = frame["x0"].astype(np.int64) + rng.integers(-3, 4, n)
    y0 = frame["y0"].astype(np.int64) + rng.integers(-3, 4, n)
    desc = np.stack([flip_bits(d, int(rng.integers(0, 40)), rng) for d in frame["desc"]])
    kr = refs(np.clip(x0, 0, None), np.clip(y0, 0, None), frame["level"], desc)
    idx, d1, d2 = oracle.feature_match(frame, kr, 8, 1, 64, 90)
    assert (idx >= 0).mean() > 0.5
    perm = rng.permutation(n)
    kp = refs(kr["x0"][perm], kr["y0"][perm], kr["level"][perm], kr["desc"][perm])
    idx2, e1, e2 = oracle.feature_match(frame, kp, 8, 1, 64, 90)
    assert np.array_equal(d1, e1) and np.array_equal(d2, e2)
    # accepted matches are unique in distance (ratio test), so the index maps
    ok = idx >= 0
    assert np.array_equal(perm[idx2[ok]], idx[ok])
