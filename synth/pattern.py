"""Seeded draws the method consumes as inputs.

* The rBRIEF test pattern: 256 point pairs inside the radius-15 disc.  ORB
  uses a learned pattern whose table is third-party data, so this project
  draws its own with BRIEF's isotropic-Gaussian sampling: each point is an
  i.i.d. N(0, (31/5)^2) draw per axis, rounded to the nearest integer and
  redrawn until it lies in u^2 + v^2 <= 225; a pair with p == q is redrawn.
* Initial CNN weights for the learned cell proposer.

Both the CPU oracle and the GPU library receive these arrays as arguments;
neither side generates them.
"""
from __future__ import annotations

import numpy as np

PATTERN_SEED = 20241004
DISC_R2 = 225


def brief_pattern(seed: int = PATTERN_SEED, n_pairs: int = 256) -> np.ndarray:
    """Return an int8 array (n_pairs, 4) of (pu, pv, qu, qv)."""
    rng = np.random.default_rng([int(seed), 11])
    sigma = 31.0 / 5.0

    def point():
        while True:
            u, v = np.rint(rng.normal(0.0, sigma, 2)).astype(np.int64)
            if u * u + v * v <= DISC_R2:
                return int(u), int(v)

    out = np.zeros((n_pairs, 4), dtype=np.int8)
    i = 0
    while i < n_pairs:
        p = point()
        q = point()
        if p == q:
            continue
        out[i] = (p[0], p[1], q[0], q[1])
        i += 1
    return out


# CNN of the learned cell proposer: 3 strided 3x3 convolutions and a 1x1 head.
CNN_CHANNELS = (1, 16, 32, 32)


def cnn_param_shapes():
    """Shapes of (w1, b1, w2, b2, w3, b3, w4, b4); weights are OIHW."""
    c0, c1, c2, c3 = CNN_CHANNELS
    return [(c1, c0, 3, 3), (c1,), (c2, c1, 3, 3), (c2,), (c3, c2, 3, 3), (c3,),
            (1, c3, 1, 1), (1,)]


def cnn_init(seed: int = 7) -> list:
    """He-normal weights, zero biases, float32."""
    rng = np.random.default_rng([int(seed), 13])
    out = []
    for shp in cnn_param_shapes():
        if len(shp) == 1:
            out.append(np.zeros(shp, dtype=np.float32))
        else:
            fan_in = shp[1] * shp[2] * shp[3]
            out.append((rng.normal(0.0, np.sqrt(2.0 / fan_in), shp)).astype(np.float32))
    return out
