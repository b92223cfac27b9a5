"""Seeded synthetic scenes with known corners, rendered at any rotation.

Input of the repeatability harness: the paper measures how well corners
survive a rotation of the scene on synthetic shapes with labelled corners
(F1 against the labels).  None of those images are available here, so a
scene is drawn as filled polygons placed one per cell of a coarse grid
inside the disc that stays in view under any rotation (so they never
overlap or leave the image), on a constant background, each with an
intensity at least 40 grey levels from the background.  Rectangles,
triangles and star-shaped polygons (3..8 vertices at sorted random angles)
alternate.  A rotation turns every vertex about the image centre; the
rotated polygons are painted with the same pixel-centre rasteriser as the
other scenes, then blurred and noised as they are.

Ground truth: the rotated vertices whose interior angle differs from a
straight angle by at least 30 degrees (a vertex on an almost straight
outline is no corner).

This module draws and paints only; it holds no arithmetic of the detector.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import scenes


@dataclass
class CornerScene:
    width: int
    height: int
    background: int
    polygons: list            # (xs, ys, value) in the unrotated frame


def corner_scene(seed: int, width: int = 480, height: int = 480, cells: int = 6) -> CornerScene:
    rng = np.random.default_rng([int(seed), 11])
    bg = int(rng.integers(0, 256))
    cx0, cy0 = width / 2.0, height / 2.0
    disc = min(width, height) / 2.0 - 12.0             # stays in view under rotation
    step = 2.0 * disc / cells
    polys = []
    k = 0
    for gy in range(cells):
        for gx in range(cells):
            cx = cx0 - disc + (gx + 0.5) * step
            cy = cy0 - disc + (gy + 0.5) * step
            r = 0.42 * step
            if np.hypot(cx - cx0, cy - cy0) + r > disc:
                continue
            while True:
                value = int(rng.integers(0, 256))
                if abs(value - bg) >= 40:
                    break
            kind = k % 3
            k += 1
            if kind == 0:                               # rectangle at a random angle
                a = rng.uniform(0, np.pi)
                hw, hh = r * rng.uniform(0.5, 0.95), r * rng.uniform(0.5, 0.95)
                loc = np.array([[-hw, -hh], [hw, -hh], [hw, hh], [-hw, hh]])
                rot = np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
                pts = loc @ rot.T
            elif kind == 1:                             # triangle
                ang = np.sort(rng.uniform(0, 2 * np.pi, 3))
                pts = np.stack([r * np.cos(ang), r * np.sin(ang)], 1)
            else:                                       # star-shaped polygon
                nv = int(rng.integers(3, 9))
                ang = np.sort(rng.uniform(0, 2 * np.pi, nv))
                rad = r * rng.uniform(0.35, 1.0, nv)
                pts = np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)
            polys.append((cx + pts[:, 0], cy + pts[:, 1], value))
    return CornerScene(width, height, bg, polys)


def _rotate(xs, ys, deg, cx, cy):
    a = np.deg2rad(deg)
    c, s = np.cos(a), np.sin(a)
    dx, dy = xs - cx, ys - cy
    return cx + c * dx - s * dy, cy + s * dx + c * dy


def interior_angles(xs, ys):
    """Interior angle (degrees) at every vertex of a simple polygon."""
    p = np.stack([xs, ys], 1)
    prev, nxt = np.roll(p, 1, 0), np.roll(p, -1, 0)
    a1 = np.arctan2(prev[:, 1] - p[:, 1], prev[:, 0] - p[:, 0])
    a2 = np.arctan2(nxt[:, 1] - p[:, 1], nxt[:, 0] - p[:, 0])
    turn = np.rad2deg((a1 - a2) % (2 * np.pi))          # angle from the next edge to the previous one
    # orientation: the interior is on the side of the polygon's signed area
    area = 0.5 * np.sum(xs * np.roll(ys, -1) - np.roll(xs, -1) * ys)
    return turn if area > 0 else 360.0 - turn


def render_rotated(sc: CornerScene, deg: float, noise_seed, blur_sigma: float = 1.0, noise_sigma: float = 3.0):
    """(uint8 image, ground-truth corners (n, 2) as (x, y)) of the scene rotated by `deg` degrees."""
    cx, cy = sc.width / 2.0, sc.height / 2.0
    canvas = np.full((sc.height, sc.width), float(sc.background), dtype=np.float32)
    gt = []
    for xs, ys, value in sc.polygons:
        rx, ry = _rotate(xs, ys, deg, cx, cy)
        scenes._paint_poly(canvas, scenes.Polygon(rx, ry, False, value, 0), 0.0)
        ang = interior_angles(rx, ry)
        keep = np.abs(ang - 180.0) >= 30.0
        # vertex (x, y) in continuous coordinates; pixel centres sit at +0.5
        gt.append(np.stack([rx[keep] - 0.5, ry[keep] - 0.5], 1))
    img = scenes.finish(canvas, noise_seed, blur_sigma, noise_sigma)
    return img, (np.concatenate(gt) if gt else np.zeros((0, 2)))
