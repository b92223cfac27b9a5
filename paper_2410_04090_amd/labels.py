"""Training labels of the learned cell proposer (host side).

A native-scale cell is positive when a final keypoint of the exact path
(any level) has its native-scale position (x0, y0) inside it.  Each
stride-8 grid position of level 3 takes the label of the cell containing
its projected centre, x0 = min(((8 j + 4) S_3 + 2^15) >> 16, W - 1), the
same projection the library's cnn_propose uses.
"""
from __future__ import annotations

import numpy as np

S3 = (2 * 65536 * 216 + 125) // 250          # round(65536 * 1.2^3)


def grid_shape(w3: int, h3: int):
    wz, hz = w3, h3
    for _ in range(3):
        wz, hz = (wz + 1) // 2, (hz + 1) // 2
    return wz, hz


def positive_cells(x0, y0, W: int, H: int, cell0: int = 32) -> np.ndarray:
    ncx, ncy = -(-W // cell0), -(-H // cell0)
    lab = np.zeros((ncy, ncx), np.uint8)
    if len(x0):
        lab[np.asarray(y0, np.int64) // cell0, np.asarray(x0, np.int64) // cell0] = 1
    return lab


def grid_cell_index(W: int, H: int, wz: int, hz: int, cell0: int = 32):
    cols = np.minimum(((8 * np.arange(wz, dtype=np.int64) + 4) * S3 + 32768) >> 16, W - 1) // cell0
    rows = np.minimum(((8 * np.arange(hz, dtype=np.int64) + 4) * S3 + 32768) >> 16, H - 1) // cell0
    return rows, cols


def grid_targets(lab: np.ndarray, W: int, H: int, wz: int, hz: int, cell0: int = 32) -> np.ndarray:
    rows, cols = grid_cell_index(W, H, wz, hz, cell0)
    return lab[rows[:, None], cols[None, :]].astype(np.float32)


def contrast_scores(level3: np.ndarray, W: int, H: int, cell0: int = 32) -> np.ndarray:
    """Non-learned baseline proposer: per native-scale cell, the intensity
    range (max - min) of level 3 over the cell's footprint, widened by the
    3-pixel ring radius."""
    h3, w3 = level3.shape
    ncx, ncy = -(-W // cell0), -(-H // cell0)
    out = np.zeros((ncy, ncx), np.float32)
    s = S3 / 65536.0
    for cy in range(ncy):
        y0 = max(int(cy * cell0 / s) - 3, 0)
        y1 = min(int(-(-((cy + 1) * cell0) // s)) + 3, h3)
        for cx in range(ncx):
            x0 = max(int(cx * cell0 / s) - 3, 0)
            x1 = min(int(-(-((cx + 1) * cell0) // s)) + 3, w3)
            blk = level3[y0:y1, x0:x1]
            out[cy, cx] = float(blk.max()) - float(blk.min()) if blk.size else 0.0
    return out
