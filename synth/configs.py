"""The five synthetic workloads and their pipeline parameters.

Each workload lists the images it is made of (size, seed, scene density,
disparity range) and the parameter set of the front-end run on it.
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict, replace

import numpy as np

from . import scenes


@dataclass(frozen=True)
class Params:
    eps_hi: int = 20        # FAST intensity threshold
    eps_lo: int = 7         # per-cell fallback threshold, -1 = none
    p_min: int = 9          # shortest accepted contiguous run
    p_max: int = 13         # Bounded Rectification upper bound (16 = plain FAST)
    border: int = 16        # pixels skipped at each level edge
    n_levels: int = 8       # pyramid levels at scale 6/5
    cell0: int = 32         # level-0 cell size
    pfa: int = 1            # pyramidal feature aggregation on/off
    nms_mode: int = 0       # 0 = lexicographic (k_l, k_r), 1 = both strictly larger
    nms_radius: int = 1     # NMS window q = 2 r + 1 at the native scale
    n_max: int = 2000       # keypoints kept per image
    blur: int = 1           # smooth before rBRIEF sampling
    d_max: int = 96         # stereo disparity search range at level 0
    match_th: int = 64      # largest accepted Hamming distance
    row_band: int = 1       # |dy| tolerance in level pixels

    def as_dict(self):
        return asdict(self)


@dataclass
class Workload:
    name: str
    sizes: list                  # [(W, H)] per stereo pair (or per mono image)
    seeds: list
    params: Params
    stereo: bool = True
    n_polygons: int = 200
    max_disparity: int = 64
    describe: bool = True        # run orientation + rBRIEF + matching
    extra: dict = field(default_factory=dict)

    @property
    def n_images(self) -> int:
        return len(self.sizes) * (2 if self.stereo else 1)

    def image_sizes(self):
        out = []
        for (w, h) in self.sizes:
            out.append((w, h))
            if self.stereo:
                out.append((w, h))
        return out

    def images(self):
        """List of uint8 arrays: left, right, left, right, ... (or mono)."""
        out = []
        for (w, h), s in zip(self.sizes, self.seeds):
            if self.stereo:
                left, right = scenes.stereo_pair(s, w, h, self.n_polygons, self.max_disparity)
                out += [left, right]
            else:
                out.append(scenes.mono_image(s, w, h, self.n_polygons))
        return out


def mono_752x480() -> Workload:
    """Single 752x480 image, one level, FAST-9 eps 20 with BR, 32x32 cells."""
    p = Params(eps_hi=20, eps_lo=-1, border=3, n_levels=1, pfa=0, n_max=4096,
               blur=0, d_max=0)
    return Workload("mono_752x480_L1", [(752, 480)], [1], p, stereo=False,
                    describe=False)


def pair_1241x376() -> Workload:
    """One rectified 1241x376 pair through the full 8-level pipeline."""
    return Workload("pair_1241x376_L8", [(1241, 376)], [2], Params())


def batch32_mixed() -> Workload:
    """32 pairs, 8 each of 640x480, 752x480, 1241x376, 1280x720."""
    sizes = [(640, 480)] * 8 + [(752, 480)] * 8 + [(1241, 376)] * 8 + [(1280, 720)] * 8
    return Workload("batch32_mixed_L8", sizes, list(range(100, 132)), Params())


def learned_1241x376() -> Workload:
    """Learned-proposal evaluation pairs at 1241x376 (held-out seeds)."""
    return Workload("learned_1241x376_L8", [(1241, 376)] * 8,
                    [2_000_000 + i for i in range(8)], Params())


def batch64_1080p() -> Workload:
    """64 pairs of 1920x1080, 800 polygons, disparities 0..128."""
    p = Params(n_max=4000, d_max=128)
    return Workload("batch64_1920x1080_L8", [(1920, 1080)] * 64,
                    list(range(200, 264)), p, n_polygons=800, max_disparity=128)


WORKLOADS = {"mono_752x480": mono_752x480, "pair_1241x376": pair_1241x376, "batch32_mixed": batch32_mixed,
             "learned_1241x376": learned_1241x376, "batch64_1080p": batch64_1080p}


def small_variant(w: Workload, scale: float) -> Workload:
    """Same parameters on proportionally smaller images (for fast tests)."""
    sizes = [(max(48, int(a * scale)), max(48, int(b * scale))) for a, b in w.sizes]
    return replace(w, sizes=sizes)
