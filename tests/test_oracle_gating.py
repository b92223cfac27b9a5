"""Pins of the oracle's learned-gating footprint (``or_cell_runs``).

A level-l cell of side c at (cx, cy) runs when the native-scale image of its
area overlaps a kept level-0 cell.  The oracle evaluates that as one
interval per axis, [x S >> 16, ceil((x + c) S / 2^16)), with x = cx c and
S = round(65536 * 1.2^l), then walks the level-0 cells between the floor of
the start and the ceiling of the end.  The brute force here takes a
different route: it maps every pixel square [x, x + 1) of the cell to
[x S, (x + 1) S) / 2^16 at the native scale and lists, pixel by pixel, the
level-0 cells [32 a, 32 a + 32) that this span overlaps with positive
length (integer comparisons only, no floor or ceiling).  Random partial
masks then have to give the same run flag for every cell of every level.

A second check pins the purpose of the rule: the aggregation step projects
a level-l keypoint to x0 = min((x S + 2^15) >> 16, W - 1); every pixel
whose projection lands in a kept level-0 cell belongs to a running cell, so
gating never drops a keypoint that a perfect proposer would keep.
"""
import numpy as np
import pytest

import oracle

CELL0 = 32


def pixel_cells(c, n_cells_l, S, ncx0):
    """Per level-l cell index along one axis: the level-0 cells overlapped
    by the native span of any of its pixels (pixel by pixel)."""
    out = []
    for k in range(n_cells_l):
        cells = set()
        for x in range(k * c, k * c + c):
            lo, hi = x * S, (x + 1) * S          # native span of the pixel, times 2^16
            # candidate cells: a loose window around the pixel (the integer
            # comparisons below decide)
            near = lo // (CELL0 * 65536)
            for a in range(max(near - 2, 0), min(near + 3, ncx0)):
                if (CELL0 * a) * 65536 < hi and (CELL0 * a + CELL0) * 65536 > lo:
                    cells.add(a)
        out.append(sorted(cells))
    return out


# (the wide images reach the cell boundaries where the end of a footprint
# lies less than half a pixel past a level-0 cell edge: a rounded instead of
# a ceiled end differs only there)
@pytest.mark.parametrize("W,H", [(1241, 376), (640, 480), (1920, 1080), (333, 201), (97, 61), (8192, 48),
                                 (48, 8192), (5000, 40)])
def test_cell_runs_matches_pixel_brute_force(W, H):
    rng = np.random.default_rng(W * 7 + H)
    ncx0, ncy0 = -(-W // CELL0), -(-H // CELL0)
    masks = [(rng.random((ncy0, ncx0)) < q).astype(np.uint8) for q in (0.1, 0.3, 0.5, 0.7)]
    # a mask with a single kept cell exposes every boundary of its neighbours
    one = np.zeros((ncy0, ncx0), np.uint8)
    one[ncy0 // 2, ncx0 // 2] = 1
    masks.append(one)
    outcomes = {True: 0, False: 0}
    for l in range(1, 8):
        w, h = oracle.level_size(W, H, l)
        c = oracle.cell_size(CELL0, l)
        S = int(oracle.scale_q16(l))
        ncx, ncy = -(-w // c), -(-h // c)
        ax = pixel_cells(c, ncx, S, ncx0)
        ay = pixel_cells(c, ncy, S, ncy0)
        for m in masks:
            for cy in range(ncy):
                for cx in range(ncx):
                    ref = bool(m[np.ix_(ay[cy], ax[cx])].any()) if ay[cy] and ax[cx] else False
                    got = oracle.cell_runs(l, cx, cy, c, W, H, CELL0, m)
                    assert got == ref, (W, H, l, cx, cy, ax[cx], ay[cy])
                    outcomes[got] += 1
    # the masks are partial: both outcomes occur many times
    assert min(outcomes.values()) >= 20, outcomes


@pytest.mark.parametrize("W,H", [(1241, 376), (640, 480)])
def test_projection_of_every_pixel_lies_in_its_cells_footprint(W, H):
    ncx0, ncy0 = -(-W // CELL0), -(-H // CELL0)
    for l in range(1, 8):
        w, h = oracle.level_size(W, H, l)
        c = oracle.cell_size(CELL0, l)
        S = int(oracle.scale_q16(l))
        ncx, ncy = -(-w // c), -(-h // c)
        for axis, n_l, lim, nc in ((0, w, W, ncx), (1, h, H, ncy)):
            pos = np.arange(n_l, dtype=np.int64)
            x0 = np.minimum((pos * S + 32768) >> 16, lim - 1)
            cell0 = x0 // CELL0
            for k in range(nc):
                # only the projected cell is kept: the pixel's cell must run
                for x in range(k * c, min(k * c + c, n_l)):
                    if axis == 0:
                        m = np.zeros((ncy0, ncx0), np.uint8)
                        m[:, cell0[x]] = 1
                        assert oracle.cell_runs(l, k, 0, c, W, H, CELL0, m), (l, k, x)
                    else:
                        m = np.zeros((ncy0, ncx0), np.uint8)
                        m[cell0[x], :] = 1
                        assert oracle.cell_runs(l, 0, k, c, W, H, CELL0, m), (l, k, x)


def test_all_and_none():
    m1 = np.ones((12, 39), np.uint8)
    m0 = np.zeros((12, 39), np.uint8)
    for l in range(8):
        c = oracle.cell_size(CELL0, l)
        w, h = oracle.level_size(1241, 376, l)
        for cy in range(-(-h // c)):
            for cx in range(-(-w // c)):
                assert oracle.cell_runs(l, cx, cy, c, 1241, 376, CELL0, m1)
                assert not oracle.cell_runs(l, cx, cy, c, 1241, 376, CELL0, m0)
