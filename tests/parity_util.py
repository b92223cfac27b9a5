"""Helpers of the GPU parity tests: run the HIP path and the oracle on the
same seeded bytes and compare every stage element by element."""
from __future__ import annotations

import sys

import numpy as np

import oracle

KEY_FALLBACK = 1 << 22


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_image(img, params, pattern, mask0=None):
    """Oracle pyramid (packed), keypoints with descriptors."""
    H, W = img.shape
    packed = oracle.pyramid_packed(img, params.n_levels)
    kps = oracle.detect(packed, W, H, params, mask0)
    if params.border >= 15:
        kps = oracle.describe(packed, W, H, params, pattern, kps)
    return packed, kps


def compare_pyramid(fe, i, img, params):
    H, W = img.shape
    ref = oracle.pyramid(img, params.n_levels)
    got = fe.pyramid_levels(i)
    for l, (a, b) in enumerate(zip(ref, got)):
        assert a.shape == b.shape, (i, l, a.shape, b.shape)
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            raise AssertionError("pyramid image %d level %d: %d px differ, first %s ref %d got %d"
                                 % (i, l, len(bad), bad[0], a[tuple(bad[0])], b[tuple(bad[0])]))
    return ref


def compare_cells(fe, i, levels, params):
    for l, lvl in enumerate(levels):
        c = oracle.cell_size(params.cell0, l)
        key, flag = oracle.cull_level(lvl, c, params)
        ref = key.astype(np.uint64) | (flag.astype(np.uint64) << 22)
        got = fe.cell_keys_level(i, l).astype(np.uint64)
        if not np.array_equal(ref, got):
            bad = np.argwhere(ref != got)
            raise AssertionError("cell keys image %d level %d: %d differ, first %s ref %x got %x"
                                 % (i, l, len(bad), bad[0], int(ref[tuple(bad[0])]), int(got[tuple(bad[0])])))


def compare_crf(fe, i, levels, params):
    for l, lvl in enumerate(levels):
        ref = oracle.crf(lvl, params.eps_hi, params.p_min, params.p_max, params.border)
        got = fe.crf_level(i, l)
        assert np.array_equal(ref, got), "crf image %d level %d" % (i, l)


KP_CMP = ("x", "y", "level", "flags", "score", "x0", "y0", "kl", "kr")


def compare_kps(ref, got, i, describe=True):
    assert len(ref["x"]) == len(got["x"]), "image %d: %d vs %d keypoints" % (i, len(ref["x"]), len(got["x"]))
    for k in KP_CMP:
        a, b = np.asarray(ref[k]).astype(np.int64), np.asarray(got[k]).astype(np.int64)
        if not np.array_equal(a, b):
            j = int(np.argmax(a != b))
            raise AssertionError("image %d field %s differs at %d: ref %d got %d" % (i, k, j, a[j], b[j]))
    if describe:
        assert np.array_equal(ref["bin"].astype(np.int64), got["bin"].astype(np.int64)), "image %d bins" % i
        if not np.array_equal(ref["desc"], got["desc"]):
            j = int(np.argmax((ref["desc"] != got["desc"]).any(1)))
            raise AssertionError("image %d descriptor %d differs" % (i, j))


def compare_matches(fe, pair, kl, kr, params):
    ri, rd, rp = oracle.stereo(kl, kr, params)
    gi, gd, gp = fe.matches(pair)
    assert np.array_equal(ri, gi), "pair %d match idx" % pair
    assert np.array_equal(rd.astype(np.int64), gd.astype(np.int64)), "pair %d match dist" % pair
    assert np.array_equal(rp.astype(np.int64), gp.astype(np.int64)), "pair %d match disp" % pair
    return int((ri >= 0).sum())
