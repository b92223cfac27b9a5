"""Oracle of the learned cell proposer (test infrastructure only).

The proposer is not part of the paper; its definition:
  input   x = (I_3 - 128) / 128 on pyramid level 3 (exact in bfloat16);
  conv1   3x3, stride 2, zero padding 1, 1 -> 16 channels, ReLU;
  conv2   3x3, stride 2, zero padding 1, 16 -> 32 channels, ReLU;
  conv3   3x3, stride 2, zero padding 1, 32 -> 32 channels, ReLU;
  head    1x1, 32 -> 1: one logit per position of the stride-8 grid.
Each convolution output has ceil(in / 2) rows and columns.  Weights are
OIHW, one flat parameter vector in the order w1 b1 w2 b2 w3 b3 w4 b4.

Arithmetic is float64.  With ``bf16=True`` the weights, the input and every
stored activation are rounded to bfloat16 (round to nearest even) exactly
where the GPU stores them; sums stay float64 (the GPU accumulates in
float32), and the head output is not rounded.

Grid position (i, j) maps to the level-0 cell containing its projected
centre: x0 = min(((8 j + 4) S_3 + 32768) >> 16, W - 1), cell = x0 // cell0
(rows alike).  A cell's logit is the maximum over the positions mapped to
it; a cell with no position is always kept.
"""
from __future__ import annotations

import numpy as np

SHAPES = [(16, 1, 3, 3), (16,), (32, 16, 3, 3), (32,), (32, 32, 3, 3), (32,), (1, 32, 1, 1), (1,)]
N_PARAMS = int(sum(np.prod(s) for s in SHAPES))


def unflatten(theta):
    out, at = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[at:at + n], dtype=np.float64).reshape(s))
        at += n
    return out


def flatten(params):
    return np.concatenate([np.asarray(p, np.float64).reshape(-1) for p in params])


def bf16_round(x):
    """Round to the nearest bfloat16 value (ties to even), via float32."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def conv3x3_s2(x, w, b):
    """x (C, H, W), w (O, C, 3, 3) -> (O, ceil(H/2), ceil(W/2)), padding 1."""
    C, H, W = x.shape
    Ho, Wo = (H + 1) // 2, (W + 1) // 2
    xp = np.zeros((C, 2 * Ho + 1, 2 * Wo + 1))
    xp[:, 1:H + 1, 1:W + 1] = x
    out = np.zeros((w.shape[0], Ho, Wo))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2]          # (C, Ho, Wo)
            out += np.tensordot(w[:, :, ky, kx], patch, axes=([1], [0]))
    return out + b[:, None, None]


def conv3x3_s2_backward(x, w, g):
    """Gradients of sum(g * conv3x3_s2(x, w, b)) w.r.t. x, w, b."""
    C, H, W = x.shape
    Ho, Wo = g.shape[1:]
    xp = np.zeros((C, 2 * Ho + 1, 2 * Wo + 1))
    xp[:, 1:H + 1, 1:W + 1] = x
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2]
            gw[:, :, ky, kx] = np.tensordot(g, patch, axes=([1, 2], [1, 2]))
            gxp[:, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2] += np.tensordot(w[:, :, ky, kx], g, axes=([0], [0]))
    return gxp[:, 1:H + 1, 1:W + 1], gw, g.sum(axis=(1, 2))


def forward(level3_u8, theta, bf16=True):
    """Logits (Hz, Wz) and the cache of intermediates."""
    r = bf16_round if bf16 else (lambda v: np.asarray(v, np.float64))
    w1, b1, w2, b2, w3, b3, w4, b4 = [r(p) for p in unflatten(theta)]
    x = r((np.asarray(level3_u8, np.float64) - 128.0) / 128.0)[None]
    a1 = r(np.maximum(conv3x3_s2(x, w1, b1), 0.0))
    a2 = r(np.maximum(conv3x3_s2(a1, w2, b2), 0.0))
    a3 = r(np.maximum(conv3x3_s2(a2, w3, b3), 0.0))
    z = np.tensordot(w4[:, :, 0, 0], a3, axes=([1], [0]))[0] + b4[0]
    return z, (x, a1, a2, a3, (w1, w2, w3, w4))


def bce_with_logits(z, t, pos_weight=1.0):
    """Mean binary cross entropy and its gradient w.r.t. z."""
    z = np.asarray(z, np.float64)
    t = np.asarray(t, np.float64)
    sp_pos = np.logaddexp(0.0, -z)          # -log sigmoid(z)
    sp_neg = np.logaddexp(0.0, z)           # -log(1 - sigmoid(z))
    n = z.size
    loss = float(np.sum(pos_weight * t * sp_pos + (1 - t) * sp_neg) / n)
    s = 1.0 / (1.0 + np.exp(-z))
    g = (pos_weight * t * (s - 1.0) + (1 - t) * s) / n
    return loss, g


def backward(cache, dz):
    """Gradient of sum(dz * z) w.r.t. the flat parameter vector."""
    x, a1, a2, a3, (w1, w2, w3, w4) = cache
    gw4 = np.tensordot(dz, a3, axes=([0, 1], [1, 2])).reshape(1, 32, 1, 1)
    gb4 = np.array([dz.sum()])
    ga3 = w4[0, :, 0, 0][:, None, None] * dz[None]
    g3 = ga3 * (a3 > 0)
    ga2, gw3, gb3 = conv3x3_s2_backward(a2, w3, g3)
    g2 = ga2 * (a2 > 0)
    ga1, gw2, gb2 = conv3x3_s2_backward(a1, w2, g2)
    g1 = ga1 * (a1 > 0)
    _, gw1, gb1 = conv3x3_s2_backward(x, w1, g1)
    return flatten([gw1, gb1, gw2, gb2, gw3, gb3, gw4, gb4])


def grid_cells(W0, H0, Wz, Hz, cell0=32):
    """Level-0 cell (cy, cx) of every grid position, from its projected centre."""
    S3 = (2 * 65536 * 6 ** 3 + 5 ** 3) // (2 * 5 ** 3)        # round(65536 * 1.2^3)
    j = np.arange(Wz, dtype=np.int64)
    i = np.arange(Hz, dtype=np.int64)
    x0 = np.minimum(((8 * j + 4) * S3 + 32768) >> 16, W0 - 1)
    y0 = np.minimum(((8 * i + 4) * S3 + 32768) >> 16, H0 - 1)
    return y0 // cell0, x0 // cell0


def cell_logits(z, W0, H0, cell0=32):
    """Per level-0 cell: max logit of its mapped positions (+inf if none)."""
    Hz, Wz = z.shape
    ncx, ncy = (W0 + cell0 - 1) // cell0, (H0 + cell0 - 1) // cell0
    cy, cx = grid_cells(W0, H0, Wz, Hz, cell0)
    out = np.full((ncy, ncx), -np.inf)
    for a in range(Hz):
        for b in range(Wz):
            out[cy[a], cx[b]] = max(out[cy[a], cx[b]], z[a, b])
    out[np.isneginf(out)] = np.inf
    return out


def cell_targets(kp_x0, kp_y0, W0, H0, cell0=32):
    """Positive level-0 cells: those holding the native-scale position of a
    final keypoint of the exact path (any level)."""
    ncx, ncy = (W0 + cell0 - 1) // cell0, (H0 + cell0 - 1) // cell0
    t = np.zeros((ncy, ncx), np.uint8)
    t[np.asarray(kp_y0, np.int64) // cell0, np.asarray(kp_x0, np.int64) // cell0] = 1
    return t


def grid_targets(cell_t, W0, H0, Wz, Hz, cell0=32):
    cy, cx = grid_cells(W0, H0, Wz, Hz, cell0)
    return cell_t[cy[:, None], cx[None, :]].astype(np.float64)
