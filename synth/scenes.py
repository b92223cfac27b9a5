"""Seeded synthetic stereo scenes.

The paper evaluates on KITTI, EuRoC and KAIST-VIO frames; none of those are
available here, so every input is generated: a constant background, a set of
filled polygons (half axis-aligned rectangles, half star-shaped polygons),
a float Gaussian blur and additive Gaussian noise, clipped to uint8.  A
rectified right view is the same scene with each polygon shifted left by its
own integer disparity.

This module holds no arithmetic of the detector or descriptor: it only draws
random numbers and paints pixels.  Both the CPU oracle and the GPU path read
the bytes it returns.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy import ndimage


@dataclass
class Polygon:
    xs: np.ndarray      # vertex x (float64, image pixels)
    ys: np.ndarray      # vertex y
    rect: bool          # axis-aligned rectangle (fast path when painting)
    value: int          # intensity 0..255
    disparity: int      # integer disparity in pixels (right view shifts by -d)


@dataclass
class Scene:
    width: int
    height: int
    background: int
    polygons: list


def make_scene(seed: int, width: int, height: int, n_polygons: int = 200,
               max_disparity: int = 64) -> Scene:
    """Draw the geometry of one scene from ``seed``.

    Centres are uniform over the image, radii uniform in [6, min(W, H) / 6],
    intensities uniform in 0..255 and disparities uniform in 0..max_disparity.
    Even-indexed polygons are rectangles, odd-indexed ones are star-shaped
    polygons with 3..8 vertices at sorted random angles.
    """
    rng = np.random.default_rng([int(seed), 0])
    bg = int(rng.integers(0, 256))
    rmax = max(6.0, min(width, height) / 6.0)
    polys = []
    for i in range(n_polygons):
        cx = rng.uniform(0.0, width)
        cy = rng.uniform(0.0, height)
        r = rng.uniform(6.0, rmax)
        value = int(rng.integers(0, 256))
        disp = int(rng.integers(0, max_disparity + 1))
        if i % 2 == 0:
            hw = r * rng.uniform(0.4, 1.0)
            hh = r * rng.uniform(0.4, 1.0)
            xs = np.array([cx - hw, cx + hw, cx + hw, cx - hw])
            ys = np.array([cy - hh, cy - hh, cy + hh, cy + hh])
            polys.append(Polygon(xs, ys, True, value, disp))
        else:
            nv = int(rng.integers(3, 9))
            ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, nv))
            rad = r * rng.uniform(0.35, 1.0, nv)
            xs = cx + rad * np.cos(ang)
            ys = cy + rad * np.sin(ang)
            polys.append(Polygon(xs, ys, False, value, disp))
    return Scene(width, height, bg, polys)


def _paint_rect(canvas: np.ndarray, p: Polygon, dx: float) -> None:
    h, w = canvas.shape
    # a pixel is inside when its centre (x + 0.5, y + 0.5) lies in [x0, x1) x [y0, y1)
    x0 = int(np.ceil(p.xs.min() + dx - 0.5))
    x1 = int(np.ceil(p.xs.max() + dx - 0.5))
    y0 = int(np.ceil(p.ys.min() - 0.5))
    y1 = int(np.ceil(p.ys.max() - 0.5))
    x0, x1 = max(x0, 0), min(x1, w)
    y0, y1 = max(y0, 0), min(y1, h)
    if x0 < x1 and y0 < y1:
        canvas[y0:y1, x0:x1] = p.value


def _paint_poly(canvas: np.ndarray, p: Polygon, dx: float) -> None:
    """Even-odd scanline fill sampled at pixel centres."""
    h, w = canvas.shape
    xs = p.xs + dx
    ys = p.ys
    bx0 = max(int(np.floor(xs.min())), 0)
    bx1 = min(int(np.ceil(xs.max())) + 1, w)
    by0 = max(int(np.floor(ys.min())), 0)
    by1 = min(int(np.ceil(ys.max())) + 1, h)
    if bx0 >= bx1 or by0 >= by1:
        return
    yc = np.arange(by0, by1, dtype=np.float64)[:, None] + 0.5      # (R, 1)
    ax, ay = xs[None, :], ys[None, :]
    bxv, byv = np.roll(xs, -1)[None, :], np.roll(ys, -1)[None, :]
    crosses = ((ay <= yc) & (yc < byv)) | ((byv <= yc) & (yc < ay))
    with np.errstate(divide="ignore", invalid="ignore"):
        xc = ax + (yc - ay) * (bxv - ax) / (byv - ay)
    # first pixel whose centre lies right of the crossing
    t = np.floor(xc + 0.5)
    t = np.where(crosses, t, np.inf)
    t = np.clip(t, bx0, bx1) - bx0                                   # inf -> bx1-bx0 (dropped)
    ncol = bx1 - bx0
    tog = np.zeros((by1 - by0, ncol + 1), dtype=np.int32)
    rows = np.broadcast_to(np.arange(by1 - by0)[:, None], t.shape)
    np.add.at(tog, (rows[crosses], t[crosses].astype(np.int64)), 1)
    inside = (np.cumsum(tog[:, :ncol], axis=1) & 1).astype(bool)
    sub = canvas[by0:by1, bx0:bx1]
    sub[inside] = p.value


def render(scene: Scene, view: int = 0) -> np.ndarray:
    """Paint the noiseless, unblurred scene.  view 0 = left, 1 = right."""
    canvas = np.full((scene.height, scene.width), float(scene.background), dtype=np.float32)
    for p in scene.polygons:
        dx = -float(p.disparity) if view == 1 else 0.0
        if p.rect:
            _paint_rect(canvas, p, dx)
        else:
            _paint_poly(canvas, p, dx)
    return canvas


def finish(canvas: np.ndarray, noise_seed, blur_sigma: float = 1.0,
           noise_sigma: float = 3.0) -> np.ndarray:
    """Gaussian blur (radius 4 sigma), additive noise, round, clip to uint8."""
    img = canvas
    if blur_sigma > 0:
        img = ndimage.gaussian_filter(img, sigma=blur_sigma, truncate=4.0, mode="nearest")
    if noise_sigma > 0:
        rng = np.random.default_rng(noise_seed)
        img = img + rng.normal(0.0, noise_sigma, img.shape).astype(np.float32)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def mono_image(seed: int, width: int, height: int, n_polygons: int = 200,
               blur_sigma: float = 1.0, noise_sigma: float = 3.0) -> np.ndarray:
    sc = make_scene(seed, width, height, n_polygons)
    return finish(render(sc, 0), [int(seed), 1], blur_sigma, noise_sigma)


def stereo_pair(seed: int, width: int, height: int, n_polygons: int = 200,
                max_disparity: int = 64, blur_sigma: float = 1.0,
                noise_sigma: float = 3.0):
    """Return (left, right) uint8 images of one rectified pair."""
    sc = make_scene(seed, width, height, n_polygons, max_disparity)
    left = finish(render(sc, 0), [int(seed), 1], blur_sigma, noise_sigma)
    right = finish(render(sc, 1), [int(seed), 2], blur_sigma, noise_sigma)
    return left, right


def random_image(seed: int, width: int, height: int) -> np.ndarray:
    """I.i.d. uniform bytes: a dense-corner stress input for parity tests."""
    rng = np.random.default_rng([int(seed), 7])
    return rng.integers(0, 256, (height, width), dtype=np.uint8)
