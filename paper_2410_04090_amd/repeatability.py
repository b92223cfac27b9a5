"""Repeatability of FAST corners under rotation, with and without Bounded
Rectification: the paper's evidence for Sec. II-A (Eq. 1-3), an F1 score
against labelled corners of synthetic shapes as the scene rotates
(Sec. IV-A, repeatability figure).

Detections of one detector on one image: the pixels with a non-zero
single-level response (the library's fast_br_detect response dump at
threshold eps, one pyramid level, no culling), thinned by 3 x 3
non-maximum suppression on the response: a pixel survives when no
neighbour has a larger response, nor the same response earlier in raster
order.  Bounded Rectification is p_max = 13, plain FAST-9 p_max = 16.

Score: detections and ground-truth corners are paired greedily by
increasing distance (ties by detection, then corner order), one to one,
within `tol` pixels; precision = pairs / detections, recall = pairs /
corners, F1 = 2 P R / (P + R) (0 when there is no pair).

Scenes: synth.corners (polygons whose vertices are the labels).
"""
from __future__ import annotations

import numpy as np

ANGLES = tuple(range(-175, 176, 25))         # the paper's rotation angles (degrees)


def nms3(resp: np.ndarray):
    """(ys, xs) of the 3 x 3 maxima of a response map (ties: the first in
    raster order survives)."""
    r = np.asarray(resp, np.int64)
    H, W = r.shape
    pad = np.full((H + 2, W + 2), -1, np.int64)
    pad[1:-1, 1:-1] = r
    keep = r > 0
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            nb = pad[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
            earlier = dy < 0 or (dy == 0 and dx < 0)
            keep &= (r >= nb) if not earlier else (r > nb)
    ys, xs = np.nonzero(keep)
    return ys, xs


def match_f1(det_xy: np.ndarray, gt_xy: np.ndarray, tol: float):
    """Greedy one-to-one pairing within tol: dict(tp, n_det, n_gt, precision, recall, f1)."""
    det = np.asarray(det_xy, np.float64).reshape(-1, 2)
    gt = np.asarray(gt_xy, np.float64).reshape(-1, 2)
    nd, ng = len(det), len(gt)
    tp = 0
    if nd and ng:
        d = np.hypot(det[:, None, 0] - gt[None, :, 0], det[:, None, 1] - gt[None, :, 1])
        ii, jj = np.nonzero(d <= tol)
        order = np.lexsort((jj, ii, d[ii, jj]))
        used_d = np.zeros(nd, bool)
        used_g = np.zeros(ng, bool)
        for k in order:
            a, b = ii[k], jj[k]
            if not used_d[a] and not used_g[b]:
                used_d[a] = used_g[b] = True
                tp += 1
    p = tp / nd if nd else 0.0
    r = tp / ng if ng else 0.0
    f1 = 2 * p * r / (p + r) if tp else 0.0
    return {"tp": tp, "n_det": nd, "n_gt": ng, "precision": p, "recall": r, "f1": f1}


def scene_images(seeds, angles=ANGLES, size=480):
    """Rendered rotations of each seeded scene: list of (seed, angle, image, corners)."""
    from synth import corners
    out = []
    for s in seeds:
        sc = corners.corner_scene(s, size, size)
        for a in angles:
            img, gt = corners.render_rotated(sc, a, [int(s), 1000 + int(a) + 180])
            out.append((s, a, img, gt))
    return out


def responses_gpu(images, eps, p_max, stream=None):
    """Single-level response dumps of the library's detector for a list of same-size images."""
    import torch

    from synth.configs import Params

    from .frontend import Frontend
    h, w = images[0].shape
    p = Params(eps_hi=eps, eps_lo=-1, p_min=9, p_max=p_max, border=3, n_levels=1, pfa=0, n_max=4096, blur=0)
    fe = Frontend(p, [(w, h)] * len(images), _pattern(), with_crf=True)
    try:
        fe.upload(images)
        fe.run(describe=False, stream=stream)
        torch.cuda.synchronize()
        return [fe.crf_level(i, 0).copy() for i in range(len(images))]
    finally:
        fe.close()


def _pattern():
    from synth import pattern
    return pattern.brief_pattern()


def evaluate(cases, responses_br, responses_plain, tol=3.0):
    """Per angle: mean F1 (and precision, recall) over the scenes for both detectors."""
    rows = {}
    for (s, a, img, gt), rb, rp in zip(cases, responses_br, responses_plain):
        for name, resp in (("br", rb), ("plain", rp)):
            ys, xs = nms3(resp)
            m = match_f1(np.stack([xs, ys], 1), gt, tol)
            rows.setdefault(a, {}).setdefault(name, []).append(m)
    out = {}
    for a in sorted(rows):
        out[a] = {name: {k: float(np.mean([m[k] for m in ms])) for k in ("f1", "precision", "recall")}
                  for name, ms in rows[a].items()}
    return out


def run(seeds=(1, 2, 3, 4), angles=ANGLES, size=480, eps=20, tol=3.0):
    """The harness on the GPU: F1 per angle for Bounded Rectification and
    plain FAST-9, and their means over the angles."""
    cases = scene_images(seeds, angles, size)
    imgs = [c[2] for c in cases]
    rb = responses_gpu(imgs, eps, 13)
    rp = responses_gpu(imgs, eps, 16)
    per = evaluate(cases, rb, rp, tol)
    mean = {name: float(np.mean([per[a][name]["f1"] for a in per])) for name in ("br", "plain")}
    return {"per_angle": per, "mean_f1": mean, "scenes": len(seeds), "angles": list(angles), "size": size,
            "eps": eps, "tol_px": tol}
