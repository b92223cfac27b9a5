"""Batch front-end: owns the library context, the batch object and the
device buffers, and issues the five C-ABI calls on one stream.

Memory comes from PyTorch (device tensors); every computation is a kernel
of libvsfe.so.  ``run()`` only launches kernels, so it can be captured into
a HIP graph (``capture()`` / ``replay()``).
"""
from __future__ import annotations

import numpy as np
import torch

from . import vsfe


def _round_up(v, a):
    return (v + a - 1) // a * a


class Frontend:
    def __init__(self, params, sizes, pattern, device="cuda", tile=None, with_crf=False,
                 with_mask=False, layout=None):
        """layout: None (64-byte pitches, 256-byte image offsets: every row
        16-byte aligned) or (pitches, offsets) of the input buffer."""
        self.params = vsfe.make_params(params)
        self.sizes = [(int(w), int(h)) for (w, h) in sizes]
        self.n = len(self.sizes)
        self.device = torch.device(device)
        self.ctx = vsfe.ctx_create(self.params, pattern)
        if tile is not None:
            vsfe.ctx_set_tile(self.ctx, *tile)
        if layout is None:
            self.pitches = [_round_up(w, 64) for (w, _) in self.sizes]
            self.offsets, at = [], 0
            for (w, h), pt in zip(self.sizes, self.pitches):
                self.offsets.append(at)
                at = _round_up(at + pt * h, 256)
        else:
            self.pitches = [int(v) for v in layout[0]]
            self.offsets = [int(v) for v in layout[1]]
        self.batch = vsfe.batch_create(self.ctx, [w for w, _ in self.sizes], [h for _, h in self.sizes],
                                       self.pitches, self.offsets)
        info = vsfe.batch_info(self.batch)
        self.info = info
        dev = self.device
        u8 = dict(dtype=torch.uint8, device=dev)
        i32 = dict(dtype=torch.int32, device=dev)
        self.images = torch.zeros(max(info.input_bytes, 1), **u8)
        self.pyr = torch.zeros(max(info.pyr_bytes, 1), **u8)
        self.cell_keys = torch.zeros(max(info.n_cells, 1), **i32)
        self.workspace = torch.zeros(max(info.workspace_bytes, 1), **u8)
        cap = max(info.kp_capacity, 1)
        self.kps = {n: torch.zeros(cap, dtype=t, device=dev) for n, t in vsfe.KP_FIELDS}
        self.kp_count = torch.zeros(self.n, **i32)
        self.desc = torch.zeros(cap * 8, **i32)
        mcap = max(info.match_capacity, 1)
        self.match_idx = torch.zeros(mcap, **i32)
        self.match_dist = torch.zeros(mcap, dtype=torch.int16, device=dev)
        self.match_disp = torch.zeros(mcap, dtype=torch.int16, device=dev)
        self.refine_disp = torch.zeros(mcap, **i32)
        self.refine_sad = torch.zeros(mcap, **i32)
        self.status = torch.zeros(1, **i32)
        self.crf = torch.zeros(max(info.crf_elems, 1), dtype=torch.int16, device=dev) if with_crf else None
        self.cell_mask = torch.ones(max(info.n_cells0, 1), **u8) if with_mask else None
        self.cnn = None
        if self.params.n_levels >= 4:
            ci = vsfe.cnn_info(self.batch)
            self.cnn = ci
            self.cnn_ws = torch.zeros(max(ci.workspace_bytes, 1), **u8)
            self.grid_logits = torch.zeros(max(ci.grid_elems, 1), dtype=torch.float32, device=dev)
            self.cell_logits = torch.zeros(max(ci.n_cells0, 1), dtype=torch.float32, device=dev)
            if self.cell_mask is None:
                self.cell_mask = torch.ones(max(info.n_cells0, 1), **u8)
        self.describe = True
        self.stereo = self.n % 2 == 0 and all(self.sizes[i] == self.sizes[i + 1] for i in range(0, self.n, 2))
        self._graph = None
        self._side_stream = None

    # ------------------------------------------------------------ data in/out
    def pack(self, imgs) -> torch.Tensor:
        """Pack host uint8 images into one pinned host buffer (input layout)."""
        host = torch.zeros(self.images.numel(), dtype=torch.uint8, pin_memory=True)
        hv = host.numpy()
        for img, (w, h), pt, off in zip(imgs, self.sizes, self.pitches, self.offsets):
            assert img.shape == (h, w) and img.dtype == np.uint8
            hv[off:off + pt * h].reshape(h, pt)[:, :w] = img
        return host

    def upload(self, imgs):
        self.images.copy_(self.pack(imgs), non_blocking=False)

    def level_info(self, i, l):
        return vsfe.batch_level_info(self.batch, i, l)

    # ------------------------------------------------------------ pipeline
    def _side(self):
        if self._side_stream is None:
            self._side_stream = torch.cuda.Stream(device=self.device)
        return self._side_stream

    # below this many level-0 pixels in a batch the second branch's
    # synchronisation costs more than the overlap saves (one 1241 x 376 pair
    # loses about 20 us, 32 mixed pairs gain)
    OVERLAP_MIN_PIXELS = 4_000_000
    # with one pyramid launch per level, levels 1..OVERLAP_SPLIT are also
    # detected on the second stream (splits after levels 2..5 measured
    # within 4 µs of each other on 64 1080p pairs)
    OVERLAP_SPLIT = 3

    def run(self, stream=None, mask=None, describe=None, stereo=None, overlap=None):
        """The exact path.  With `overlap` (default: batches of at least
        OVERLAP_MIN_PIXELS level-0 pixels; never with a gate or a response
        dump) level-0 detection, which reads only the input, runs on a second
        stream while the pyramid is built (and, with one pyramid launch per
        level, detection of levels 1..OVERLAP_SPLIT once they are built,
        beside the later levels); the two branches join before the
        aggregation (also inside a captured graph)."""
        describe = self.describe if describe is None else describe
        stereo = self.stereo if stereo is None else stereo
        if overlap is None:
            overlap = sum(w * h for w, h in self.sizes) >= self.OVERLAP_MIN_PIXELS
        c, b = self.ctx, self.batch
        L = self.params.n_levels
        if overlap and mask is None and self.crf is None and L > 1:
            st = stream if stream is not None else torch.cuda.current_stream()
            side = self._side()
            side.wait_stream(st)
            vsfe.fast_br_detect_levels(c, b, self.images, self.pyr, None, self.cell_keys, 0, 1, self.status, side)
            if L > self.OVERLAP_SPLIT + 1 and vsfe.batch_pyramid_get(b)[0] == vsfe.PYR_LEVELS:
                # levels 1..3 are detected on the second stream too, while
                # the pyramid's later levels are built (≈ 25 µs per 1080p
                # step: the launches' ramps and tails overlap)
                k = self.OVERLAP_SPLIT
                vsfe.pyramid_build_levels(c, b, self.images, self.pyr, 1, k + 1, self.status, st)
                ev = torch.cuda.Event()
                ev.record(st)
                side.wait_event(ev)
                vsfe.fast_br_detect_levels(c, b, self.images, self.pyr, None, self.cell_keys, 1, k + 1, self.status,
                                           side)
                vsfe.pyramid_build_levels(c, b, self.images, self.pyr, k + 1, L, self.status, st)
                vsfe.fast_br_detect_levels(c, b, self.images, self.pyr, None, self.cell_keys, k + 1, L, self.status,
                                           st)
            else:
                vsfe.pyramid_build(c, b, self.images, self.pyr, self.status, st)
                vsfe.fast_br_detect_levels(c, b, self.images, self.pyr, None, self.cell_keys, 1, L, self.status, st)
            st.wait_stream(side)
        else:
            vsfe.pyramid_build(c, b, self.images, self.pyr, self.status, stream)
            vsfe.fast_br_detect(c, b, self.images, self.pyr, mask, self.cell_keys, self.crf, self.status, stream)
        vsfe.pyca_cull_aggregate(c, b, self.cell_keys, self.workspace, self.kps, self.kp_count, self.status,
                                 stream)
        if describe:
            vsfe.orb_describe(c, b, self.images, self.pyr, self.kps, self.kp_count, self.desc, self.status, stream)
            if stereo:
                vsfe.stereo_match(c, b, self.kps, self.kp_count, self.desc, self.match_idx, self.match_dist,
                                  self.match_disp, self.status, stream)

    def run_learned(self, params_bf16, thresh, stream=None, describe=None, stereo=None):
        """Learned-proposal path: pyramid, CNN cell proposal on level 3,
        detection gated to the proposed cells, then the unchanged rest."""
        describe = self.describe if describe is None else describe
        stereo = self.stereo if stereo is None else stereo
        c, b = self.ctx, self.batch
        L = self.params.n_levels
        if L > 4 and vsfe.batch_pyramid_get(b)[0] == vsfe.PYR_LEVELS:
            # levels 1..3 feed the proposer; levels 4.. are built on a second
            # stream while it runs, and the branches join before detection
            # (with the single-launch schedule the whole pyramid comes first:
            # one launch is shorter than the split's seven)
            st = stream if stream is not None else torch.cuda.current_stream()
            vsfe.pyramid_build_levels(c, b, self.images, self.pyr, 1, 4, self.status, st)
            side = self._side()
            side.wait_stream(st)
            vsfe.pyramid_build_levels(c, b, self.images, self.pyr, 4, L, self.status, side)
            vsfe.cnn_propose(c, b, self.pyr, params_bf16, thresh, self.cnn_ws, self.grid_logits, self.cell_logits,
                             self.cell_mask, self.status, st)
            st.wait_stream(side)
        else:
            vsfe.pyramid_build(c, b, self.images, self.pyr, self.status, stream)
            vsfe.cnn_propose(c, b, self.pyr, params_bf16, thresh, self.cnn_ws, self.grid_logits, self.cell_logits,
                             self.cell_mask, self.status, stream)
        vsfe.fast_br_detect(c, b, self.images, self.pyr, self.cell_mask, self.cell_keys, self.crf, self.status,
                            stream)
        vsfe.pyca_cull_aggregate(c, b, self.cell_keys, self.workspace, self.kps, self.kp_count, self.status,
                                 stream)
        if describe:
            vsfe.orb_describe(c, b, self.images, self.pyr, self.kps, self.kp_count, self.desc, self.status, stream)
            if stereo:
                vsfe.stereo_match(c, b, self.kps, self.kp_count, self.desc, self.match_idx, self.match_dist,
                                  self.match_disp, self.status, stream)

    # sub-pixel refinement window and search range (level pixels)
    REFINE_HALF_WINDOW = 5
    REFINE_RADIUS = 5

    def refine(self, stream=None, half_window=None, search_radius=None):
        """Sub-pixel refinement of the stereo matches (after run())."""
        vsfe.stereo_refine(self.ctx, self.batch, self.images, self.pyr, self.kps, self.kp_count, self.match_idx,
                           self.REFINE_HALF_WINDOW if half_window is None else half_window,
                           self.REFINE_RADIUS if search_radius is None else search_radius,
                           self.refine_disp, self.refine_sad, self.status, stream)

    def refined(self, pair):
        """(disparity in 1/256 native pixel or INT32_MIN, least SAD) per left keypoint."""
        n = int(self.kp_count[2 * pair].item())
        base = pair * self.params.n_max
        return (self.refine_disp[base:base + n].cpu().numpy(),
                self.refine_sad[base:base + n].cpu().numpy().view(np.uint32))

    def autotune(self, reps=5):
        """Pick per-level detector tiles on the uploaded batch (graphs captured
        before must be captured again)."""
        vsfe.pyramid_build(self.ctx, self.batch, self.images, self.pyr, self.status)
        rep = vsfe.batch_autotune(self.ctx, self.batch, self.images, self.pyr, self.cell_keys, self.status, reps)
        self._graph = None
        return rep.as_dict()

    def tiles(self):
        return vsfe.batch_tiles_get(self.batch, self.params.n_levels)

    def set_tiles(self, tile_w, tile_h):
        vsfe.batch_set_tiles(self.batch, tile_w, tile_h)
        self._graph = None

    def cnn_geometry(self, image):
        """(W3, H3, Wz, Hz) of one image's proposer grid."""
        li = self.level_info(image, 3)
        w3, h3 = li.width, li.height
        wz, hz = w3, h3
        for _ in range(3):
            wz, hz = (wz + 1) // 2, (hz + 1) // 2
        return w3, h3, wz, hz

    def grid_offsets(self):
        offs, at = [], 0
        for i in range(self.n):
            _, _, wz, hz = self.cnn_geometry(i)
            offs.append((at, hz, wz))
            at += wz * hz
        return offs

    def capture(self, fn=None, **kw):
        """Capture run() (or fn(stream=...)) into a HIP graph on a side stream."""
        fn = self.run if fn is None else fn
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn(stream=s, **kw)                # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            fn(stream=s, **kw)
        torch.cuda.synchronize()
        self._graph = g
        return g

    def replay(self):
        self._graph.replay()

    # ------------------------------------------------------------ results
    def results(self, image):
        """Keypoints (+ descriptors) of one image as numpy arrays (synchronises)."""
        n = int(self.kp_count[image].item())
        base = image * self.params.n_max
        out = {}
        for name, t in vsfe.KP_FIELDS:
            a = self.kps[name][base:base + n].cpu().numpy()
            if name in ("x", "y", "score", "x0", "y0"):
                a = a.view(np.uint16)
            elif name == "kr":
                a = a.view(np.uint32)
            out[name] = a
        out["desc"] = self.desc[base * 8:(base + n) * 8].cpu().numpy().view(np.uint32).reshape(n, 8)
        return out

    def matches(self, pair):
        n = int(self.kp_count[2 * pair].item())
        base = pair * self.params.n_max
        return (self.match_idx[base:base + n].cpu().numpy(),
                self.match_dist[base:base + n].cpu().numpy().view(np.uint16),
                self.match_disp[base:base + n].cpu().numpy())

    def pyramid_levels(self, image):
        """Levels 0..L-1 of one image as numpy arrays."""
        out = []
        for l in range(self.params.n_levels):
            li = self.level_info(image, l)
            src = self.images if l == 0 else self.pyr
            flat = src[li.offset:li.offset + li.pitch * li.height].cpu().numpy()
            out.append(flat.reshape(li.height, li.pitch)[:, :li.width].copy())
        return out

    def cell_keys_level(self, image, level):
        li = self.level_info(image, level)
        n = li.ncx * li.ncy
        a = self.cell_keys[li.cell_offset:li.cell_offset + n].cpu().numpy().view(np.uint32)
        return a.reshape(li.ncy, li.ncx)

    def crf_level(self, image, level):
        li = self.level_info(image, level)
        a = self.crf[li.crf_offset:li.crf_offset + li.width * li.height].cpu().numpy().view(np.uint16)
        return a.reshape(li.height, li.width)

    def close(self):
        if self.batch is not None:
            vsfe.batch_destroy(self.batch)
            self.batch = None
        if self.ctx is not None:
            vsfe.ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
