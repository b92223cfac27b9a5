"""Pins of the learned-proposer oracle: convolution against scipy, the
parameter count of the specified architecture, backward against finite
differences, bfloat16 rounding against torch, and the grid-to-cell map."""
import numpy as np
import pytest
from scipy import signal

from oracle import cnn


def test_param_count():
    # 3x3 convs 1->16, 16->32, 32->32 and a 1x1 head, with biases
    assert cnn.N_PARAMS == (16 * 9 + 16) + (32 * 16 * 9 + 32) + (32 * 32 * 9 + 32) + (32 + 1) == 14081


@pytest.mark.parametrize("H,W", [(9, 9), (10, 7), (1, 5)])
def test_conv_matches_scipy(H, W):
    rng = np.random.default_rng(H * 100 + W)
    x = rng.normal(size=(3, H, W))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    got = cnn.conv3x3_s2(x, w, b)
    assert got.shape == (4, (H + 1) // 2, (W + 1) // 2)
    for o in range(4):
        full = sum(signal.correlate2d(x[c], w[o, c], mode="same", boundary="fill") for c in range(3))
        assert np.allclose(got[o], full[::2, ::2] + b[o], atol=1e-12)


def test_backward_finite_differences():
    rng = np.random.default_rng(0)
    img = rng.integers(0, 256, (19, 23)).astype(np.uint8)
    theta = rng.normal(0, 0.3, cnn.N_PARAMS)
    z, cache = cnn.forward(img, theta, bf16=False)
    t = (rng.random(z.shape) < 0.5).astype(float)
    loss, dz = cnn.bce_with_logits(z, t, pos_weight=2.0)
    g = cnn.backward(cache, dz)

    def f(th):
        zz, _ = cnn.forward(img, th, bf16=False)
        return cnn.bce_with_logits(zz, t, pos_weight=2.0)[0]

    idx = list(rng.choice(cnn.N_PARAMS, 40, replace=False)) + [159, 160 + 4640 - 1, cnn.N_PARAMS - 1]
    for k in idx:
        e = np.zeros(cnn.N_PARAMS)
        e[k] = 1e-6
        fd = (f(theta + e) - f(theta - e)) / 2e-6
        assert abs(fd - g[k]) <= 1e-6 + 1e-5 * abs(fd), (k, fd, g[k])


def test_bce_reference_values():
    loss, g = cnn.bce_with_logits(np.zeros(4), np.array([0, 1, 0, 1]))
    assert abs(loss - np.log(2)) < 1e-15
    assert np.allclose(g, np.array([0.5, -0.5, 0.5, -0.5]) / 4)


def test_bf16_round_matches_torch():
    import torch
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.normal(0, 3, 10000), [1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 255.0 / 128]])
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(v), ref)
    # (I - 128) / 128 is exact in bfloat16
    k = np.arange(256)
    assert np.array_equal(cnn.bf16_round((k - 128) / 128.0), (k - 128) / 128.0)


def test_grid_cells_projection():
    cy, cx = cnn.grid_cells(1241, 376, 90, 28)
    assert cx[0] == ((4 * 113246 + 32768) >> 16) // 32 and cx[-1] <= (1241 - 1) // 32
    assert np.all(np.diff(cx) >= 0) and np.all(np.diff(cy) >= 0)
    z = np.arange(90 * 28, dtype=float).reshape(28, 90)
    cl = cnn.cell_logits(z, 1241, 376)
    assert cl.shape == (12, 39)
    # the logit of a cell is the last (largest) of its positions in this ramp
    assert cl[0, 0] == z[cy == 0][:, cx == 0].max()
    # every cell receives a position at this size (stride 8 at level 3 < 32)
    assert np.all(np.isfinite(cl))


def test_targets_from_keypoints():
    t = cnn.cell_targets([0, 40, 1240], [0, 33, 375], 1241, 376)
    assert t[0, 0] == 1 and t[1, 1] == 1 and t[11, 38] == 1 and t.sum() == 3
