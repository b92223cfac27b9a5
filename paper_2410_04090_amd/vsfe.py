"""Thin ctypes binding of libvsfe.so (argument marshalling only).

Every function here has the name of the C entry point it wraps and takes
torch tensors where the C call takes device pointers.  All computation
happens in the HIP kernels of the library; if the library is missing or
cannot be loaded, importing this module's functions raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvsfe.so")

OK, EINVAL, ECAPACITY, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
DEV_OVERFLOW = 1
KEY_FALLBACK = 1 << 22
MAX_LEVELS = 12


class VsfeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("vsfe error %d: %s" % (code, msg))
        self.code = code


class Params(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "eps_hi", "eps_lo", "p_min", "p_max", "border", "n_levels", "cell0", "pfa",
        "nms_mode", "nms_radius", "n_max", "blur", "d_max", "match_th", "row_band")]


KP_FIELDS = [("x", torch.int16), ("y", torch.int16), ("level", torch.uint8), ("flags", torch.uint8),
             ("score", torch.int16), ("x0", torch.int16), ("y0", torch.int16), ("kl", torch.uint8),
             ("kr", torch.int32), ("bin", torch.uint8)]


class KpSoa(C.Structure):
    _fields_ = [(n, C.c_void_p) for n, _ in KP_FIELDS]


class BatchInfo(C.Structure):
    _fields_ = [("input_bytes", C.c_int64), ("pyr_bytes", C.c_int64), ("crf_elems", C.c_int64),
                ("n_cells", C.c_int64), ("n_cells0", C.c_int64), ("kp_capacity", C.c_int64),
                ("workspace_bytes", C.c_int64), ("match_capacity", C.c_int64),
                ("n_images", C.c_int32), ("n_levels", C.c_int32), ("n_det_items", C.c_int32),
                ("reserved", C.c_int32)]


class LevelInfo(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("pitch", C.c_int32),
                ("cell", C.c_int32), ("ncx", C.c_int32), ("ncy", C.c_int32),
                ("offset", C.c_int64), ("cell_offset", C.c_int64), ("crf_offset", C.c_int64),
                ("cell0_offset", C.c_int64)]


class CnnInfo(C.Structure):
    _fields_ = [("workspace_bytes", C.c_int64), ("grid_elems", C.c_int64), ("n_cells0", C.c_int64),
                ("n_params", C.c_int32)]


class TuneReport(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("tile_w", C.c_int32 * MAX_LEVELS), ("tile_h", C.c_int32 * MAX_LEVELS),
                ("us", C.c_float * MAX_LEVELS), ("us_before", C.c_float * MAX_LEVELS),
                ("n_tried", C.c_int32 * MAX_LEVELS), ("us_worst", C.c_float * MAX_LEVELS),
                ("us_median", C.c_float * MAX_LEVELS), ("pyr_schedule", C.c_int32), ("pyr_tile_w", C.c_int32),
                ("pyr_tile_h", C.c_int32), ("pyr_us", C.c_float), ("pyr_us_before", C.c_float),
                ("pyr_us_worst", C.c_float), ("pyr_n_tried", C.c_int32)]

    def as_dict(self):
        n = self.n_levels
        return {"tile_w": list(self.tile_w[:n]), "tile_h": list(self.tile_h[:n]),
                "us": [round(x, 2) for x in self.us[:n]], "us_before": [round(x, 2) for x in self.us_before[:n]],
                "n_tried": list(self.n_tried[:n]), "us_worst": [round(x, 2) for x in self.us_worst[:n]],
                "us_median": [round(x, 2) for x in self.us_median[:n]],
                "pyramid": {"schedule": {PYR_LEVELS: "levels", PYR_TOWER: "tower"}.get(self.pyr_schedule, "none"),
                            "tile": [self.pyr_tile_w, self.pyr_tile_h], "us": round(self.pyr_us, 2),
                            "us_before": round(self.pyr_us_before, 2), "us_worst": round(self.pyr_us_worst, 2),
                            "n_tried": self.pyr_n_tried}}


EXPORTS = ["vsfe_params_default", "vsfe_params_check", "vsfe_level_geometry", "vsfe_ctx_create",
           "vsfe_ctx_destroy", "vsfe_batch_create", "vsfe_batch_destroy", "vsfe_batch_plan",
           "vsfe_batch_info_get", "vsfe_batch_level_info", "vsfe_ctx_set_tile", "vsfe_last_error",
           "pyramid_build", "fast_br_detect", "fast_br_detect_levels", "pyca_cull_aggregate", "orb_describe",
           "stereo_match", "vsfe_cnn_info_get", "cnn_forward", "cnn_propose", "cnn_backward", "cnn_adam_step",
           "vsfe_batch_tiles_get", "vsfe_batch_set_tiles", "vsfe_batch_autotune", "pyca_cull_aggregate_noalloc",
           "stereo_refine", "vsfe_feature_match_workspace", "feature_match",
           "vsfe_fc_cull_stride", "fc_cull_crf", "pyramid_build_levels", "vsfe_batch_set_pyramid",
           "vsfe_batch_pyramid_get", "vsfe_probe"]

NOALLOC_MAX_CELLS = 1 << 22

_lib = None


def lib():
    """Load libvsfe.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libvsfe.so is not built (run __graft_entry__.build()): " + LIB_PATH)
    L = C.CDLL(LIB_PATH)
    i32, i64, vp = C.c_int32, C.c_int64, C.c_void_p
    pi32, pi64 = C.POINTER(i32), C.POINTER(i64)
    L.vsfe_params_default.argtypes = [C.POINTER(Params)]
    L.vsfe_params_default.restype = None
    L.vsfe_params_check.argtypes = [C.POINTER(Params)]
    L.vsfe_params_check.restype = i32
    L.vsfe_level_geometry.argtypes = [C.POINTER(Params), i32, i32, i32, pi32, pi32, pi32]
    L.vsfe_level_geometry.restype = i32
    L.vsfe_ctx_create.argtypes = [C.POINTER(Params), vp, C.POINTER(vp)]
    L.vsfe_ctx_create.restype = i32
    L.vsfe_ctx_destroy.argtypes = [vp]
    L.vsfe_ctx_destroy.restype = i32
    L.vsfe_ctx_set_tile.argtypes = [vp, i32, i32]
    L.vsfe_ctx_set_tile.restype = i32
    L.vsfe_batch_create.argtypes = [vp, i32, pi32, pi32, pi32, pi64, C.POINTER(vp)]
    L.vsfe_batch_create.restype = i32
    L.vsfe_batch_plan.argtypes = [C.POINTER(Params), i32, pi32, pi32, pi32, pi64, C.POINTER(BatchInfo)]
    L.vsfe_batch_plan.restype = i32
    L.vsfe_batch_destroy.argtypes = [vp]
    L.vsfe_batch_destroy.restype = i32
    L.vsfe_batch_info_get.argtypes = [vp, C.POINTER(BatchInfo)]
    L.vsfe_batch_info_get.restype = i32
    L.vsfe_batch_level_info.argtypes = [vp, i32, i32, C.POINTER(LevelInfo)]
    L.vsfe_batch_level_info.restype = i32
    L.vsfe_batch_tiles_get.argtypes = [vp, pi32, pi32]
    L.vsfe_batch_tiles_get.restype = i32
    L.vsfe_batch_set_tiles.argtypes = [vp, pi32, pi32]
    L.vsfe_batch_set_tiles.restype = i32
    L.vsfe_probe.argtypes = [i32, i32, i32, vp, vp, vp]
    L.vsfe_probe.restype = i32
    L.vsfe_batch_set_pyramid.argtypes = [vp, i32, i32, i32]
    L.vsfe_batch_set_pyramid.restype = i32
    L.vsfe_batch_pyramid_get.argtypes = [vp, pi32, pi32, pi32]
    L.vsfe_batch_pyramid_get.restype = i32
    L.vsfe_batch_autotune.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, C.POINTER(TuneReport)]
    L.vsfe_batch_autotune.restype = i32
    L.vsfe_last_error.argtypes = []
    L.vsfe_last_error.restype = C.c_char_p
    L.pyramid_build.argtypes = [vp, vp, vp, vp, vp, vp]
    L.pyramid_build_levels.argtypes = [vp, vp, vp, vp, i32, i32, vp, vp]
    L.fast_br_detect.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.fast_br_detect_levels.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, vp, vp]
    L.pyca_cull_aggregate.argtypes = [vp, vp, vp, vp, C.POINTER(KpSoa), vp, vp, vp]
    L.pyca_cull_aggregate_noalloc.argtypes = [vp, vp, vp, C.POINTER(KpSoa), vp, vp, vp]
    L.orb_describe.argtypes = [vp, vp, vp, vp, C.POINTER(KpSoa), vp, vp, vp, vp]
    L.stereo_match.argtypes = [vp, vp, C.POINTER(KpSoa), vp, vp, vp, vp, vp, vp, vp]
    L.stereo_refine.argtypes = [vp, vp, vp, vp, C.POINTER(KpSoa), vp, vp, i32, i32, vp, vp, vp, vp]
    L.vsfe_feature_match_workspace.argtypes = [vp, pi64]
    L.feature_match.argtypes = [vp, vp, C.POINTER(KpSoa), vp, vp, C.POINTER(KpSoa), vp, vp, i32, i32, i32, i32, vp,
                                vp, vp, vp, vp, vp]
    L.vsfe_fc_cull_stride.argtypes = [vp, i32, i32, pi64]
    L.fc_cull_crf.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, i64, vp, vp]
    L.vsfe_cnn_info_get.argtypes = [vp, C.POINTER(CnnInfo)]
    L.cnn_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.cnn_propose.argtypes = [vp, vp, vp, vp, C.c_float, vp, vp, vp, vp, vp, vp]
    L.cnn_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_float, vp, vp, vp, vp]
    L.cnn_adam_step.argtypes = [vp, vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float, i32, vp]
    for f in ("pyramid_build", "pyramid_build_levels", "fast_br_detect", "fast_br_detect_levels", "pyca_cull_aggregate",
              "pyca_cull_aggregate_noalloc", "orb_describe",
              "stereo_match", "stereo_refine", "vsfe_feature_match_workspace", "feature_match", "vsfe_fc_cull_stride", "fc_cull_crf",
              "vsfe_cnn_info_get", "cnn_forward", "cnn_propose", "cnn_backward", "cnn_adam_step"):
        getattr(L, f).restype = i32
    _lib = L
    return L


def _check(rc):
    if rc != OK:
        raise VsfeError(rc, lib().vsfe_last_error().decode())


def _p(t):
    """Device pointer of a tensor (None -> NULL)."""
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expects a contiguous device tensor"
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def make_params(d=None, **kw) -> Params:
    p = Params()
    lib().vsfe_params_default(C.byref(p))
    src = {}
    if d is not None:
        src.update(d if isinstance(d, dict) else d.as_dict())
    src.update(kw)
    for k, _ in Params._fields_:
        if k in src:
            setattr(p, k, int(src[k]))
    return p


def params_check(p: Params):
    return lib().vsfe_params_check(C.byref(p))


def level_geometry(p: Params, W, H, level):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().vsfe_level_geometry(C.byref(p), W, H, level, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def _arrays(widths, heights, pitches, offsets):
    n = len(widths)
    return ((C.c_int32 * n)(*widths), (C.c_int32 * n)(*heights), (C.c_int32 * n)(*pitches),
            (C.c_int64 * n)(*offsets))


def batch_plan(p: Params, widths, heights, pitches, offsets) -> BatchInfo:
    info = BatchInfo()
    w, h, pt, of = _arrays(widths, heights, pitches, offsets)
    _check(lib().vsfe_batch_plan(C.byref(p), len(widths), w, h, pt, of, C.byref(info)))
    return info


def ctx_create(p: Params, pattern) -> C.c_void_p:
    import numpy as np
    pat = np.ascontiguousarray(pattern, dtype=np.int8)
    assert pat.shape == (256, 4)
    h = C.c_void_p()
    _check(lib().vsfe_ctx_create(C.byref(p), pat.ctypes.data_as(C.c_void_p), C.byref(h)))
    return h


def ctx_destroy(ctx):
    lib().vsfe_ctx_destroy(ctx)


def ctx_set_tile(ctx, tile_w, tile_h):
    _check(lib().vsfe_ctx_set_tile(ctx, tile_w, tile_h))


def batch_create(ctx, widths, heights, pitches, offsets) -> C.c_void_p:
    h = C.c_void_p()
    w, hh, pt, of = _arrays(widths, heights, pitches, offsets)
    _check(lib().vsfe_batch_create(ctx, len(widths), w, hh, pt, of, C.byref(h)))
    return h


def batch_destroy(b):
    lib().vsfe_batch_destroy(b)


def batch_info(b) -> BatchInfo:
    info = BatchInfo()
    _check(lib().vsfe_batch_info_get(b, C.byref(info)))
    return info


def batch_level_info(b, image, level) -> LevelInfo:
    li = LevelInfo()
    _check(lib().vsfe_batch_level_info(b, image, level, C.byref(li)))
    return li


def batch_tiles_get(b, n_levels):
    w, h = (C.c_int32 * MAX_LEVELS)(), (C.c_int32 * MAX_LEVELS)()
    _check(lib().vsfe_batch_tiles_get(b, w, h))
    return list(w[:n_levels]), list(h[:n_levels])


def batch_set_tiles(b, tile_w, tile_h):
    w = (C.c_int32 * MAX_LEVELS)(*tile_w)
    h = (C.c_int32 * MAX_LEVELS)(*tile_h)
    _check(lib().vsfe_batch_set_tiles(b, w, h))


PYR_AUTO, PYR_LEVELS, PYR_TOWER = 0, 1, 2
PROBE_VALU, PROBE_LDS = 1, 2


def probe(kind, blocks, iters, sink, clocks, stream=None):
    """Launch a ceiling probe (sink: blocks x 256 int32/float device tensor,
    clocks: 2 int64 device tensor)."""
    _check(lib().vsfe_probe(kind, blocks, iters, _p(sink), _p(clocks), _stream(stream)))


def batch_set_pyramid(b, schedule, tile_w=0, tile_h=0):
    _check(lib().vsfe_batch_set_pyramid(b, schedule, tile_w, tile_h))


def batch_pyramid_get(b):
    """(schedule pyramid_build uses, single-launch tile width, height)."""
    s, w, h = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().vsfe_batch_pyramid_get(b, C.byref(s), C.byref(w), C.byref(h)))
    return s.value, w.value, h.value


def batch_autotune(ctx, b, images, pyr, cell_keys, status, reps=5, stream=None) -> TuneReport:
    rep = TuneReport()
    _check(lib().vsfe_batch_autotune(ctx, b, _p(images), _p(pyr), _p(cell_keys), _p(status), reps,
                                     _stream(stream), C.byref(rep)))
    return rep


def kp_soa(kps: dict) -> KpSoa:
    s = KpSoa()
    for n, _ in KP_FIELDS:
        setattr(s, n, _p(kps[n]))
    return s


def pyramid_build(ctx, b, images, pyr, status, stream=None):
    _check(lib().pyramid_build(ctx, b, _p(images), _p(pyr), _p(status), _stream(stream)))


def pyramid_build_levels(ctx, b, images, pyr, level_begin, level_end, status, stream=None):
    _check(lib().pyramid_build_levels(ctx, b, _p(images), _p(pyr), int(level_begin), int(level_end), _p(status),
                                      _stream(stream)))


def fast_br_detect(ctx, b, images, pyr, cell_mask, cell_keys, crf_debug, status, stream=None):
    _check(lib().fast_br_detect(ctx, b, _p(images), _p(pyr), _p(cell_mask), _p(cell_keys),
                                _p(crf_debug), _p(status), _stream(stream)))


def fast_br_detect_levels(ctx, b, images, pyr, cell_mask, cell_keys, level_begin, level_end, status, stream=None):
    _check(lib().fast_br_detect_levels(ctx, b, _p(images), _p(pyr), _p(cell_mask), _p(cell_keys), int(level_begin),
                                       int(level_end), _p(status), _stream(stream)))


def pyca_cull_aggregate(ctx, b, cell_keys, workspace, kps, kp_count, status, stream=None):
    s = kp_soa(kps)
    _check(lib().pyca_cull_aggregate(ctx, b, _p(cell_keys), _p(workspace), C.byref(s), _p(kp_count),
                                     _p(status), _stream(stream)))


def pyca_cull_aggregate_noalloc(ctx, b, cell_keys, kps, kp_count, status, stream=None):
    s = kp_soa(kps)
    _check(lib().pyca_cull_aggregate_noalloc(ctx, b, _p(cell_keys), C.byref(s), _p(kp_count), _p(status),
                                             _stream(stream)))


def orb_describe(ctx, b, images, pyr, kps, kp_count, desc, status, stream=None):
    s = kp_soa(kps)
    _check(lib().orb_describe(ctx, b, _p(images), _p(pyr), C.byref(s), _p(kp_count), _p(desc),
                              _p(status), _stream(stream)))


def stereo_match(ctx, b, kps, kp_count, desc, match_idx, match_dist, match_disp, status, stream=None):
    s = kp_soa(kps)
    _check(lib().stereo_match(ctx, b, C.byref(s), _p(kp_count), _p(desc), _p(match_idx),
                              _p(match_dist), _p(match_disp), _p(status), _stream(stream)))


def stereo_refine(ctx, b, images, pyr, kps, kp_count, match_idx, half_window, search_radius, disp_q8, sad_min,
                  status, stream=None):
    s = kp_soa(kps)
    _check(lib().stereo_refine(ctx, b, _p(images), _p(pyr), C.byref(s), _p(kp_count), _p(match_idx),
                               int(half_window), int(search_radius), _p(disp_q8), _p(sad_min), _p(status),
                               _stream(stream)))


def feature_match_workspace(b) -> int:
    v = C.c_int64()
    _check(lib().vsfe_feature_match_workspace(b, C.byref(v)))
    return v.value


def feature_match(ctx, b, query, query_count, query_desc, ref, ref_count, ref_desc, radius, level_band, match_th,
                  ratio_pct, workspace, match_idx, dist1, dist2, status, stream=None):
    sq, sr = kp_soa(query), kp_soa(ref)
    _check(lib().feature_match(ctx, b, C.byref(sq), _p(query_count), _p(query_desc), C.byref(sr), _p(ref_count),
                               _p(ref_desc), int(radius), int(level_band), int(match_th), int(ratio_pct),
                               _p(workspace), _p(match_idx), _p(dist1), _p(dist2), _p(status), _stream(stream)))


def fc_cull_stride(b, level, cell) -> int:
    v = C.c_int64()
    _check(lib().vsfe_fc_cull_stride(b, int(level), int(cell), C.byref(v)))
    return v.value


def fc_cull_crf(ctx, b, crf, level, cell, scheme, n_loc, keys, status, stream=None):
    """keys: a 4-byte device tensor; its size is passed on and checked by
    the library (n_images x fc_cull_stride(b, level, cell) entries)."""
    assert keys.element_size() == 4, "keys holds uint32 entries"
    _check(lib().fc_cull_crf(ctx, b, _p(crf), int(level), int(cell), int(scheme), int(n_loc), _p(keys),
                             int(keys.numel()), _p(status), _stream(stream)))


# ------------------------------------------------------------- learned proposer
def cnn_info(b) -> CnnInfo:
    info = CnnInfo()
    _check(lib().vsfe_cnn_info_get(b, C.byref(info)))
    return info


def cnn_forward(ctx, b, pyr, params_bf16, workspace, grid_logits, status, stream=None):
    _check(lib().cnn_forward(ctx, b, _p(pyr), _p(params_bf16), _p(workspace), _p(grid_logits), _p(status),
                             _stream(stream)))


def cnn_propose(ctx, b, pyr, params_bf16, thresh, workspace, grid_logits, cell_logits, cell_mask, status,
                stream=None):
    _check(lib().cnn_propose(ctx, b, _p(pyr), _p(params_bf16), float(thresh), _p(workspace), _p(grid_logits),
                             _p(cell_logits), _p(cell_mask), _p(status), _stream(stream)))


def cnn_backward(ctx, b, pyr, params_bf16, workspace, grid_logits, grid_targets, pos_weight, grad, loss, status,
                 stream=None):
    _check(lib().cnn_backward(ctx, b, _p(pyr), _p(params_bf16), _p(workspace), _p(grid_logits), _p(grid_targets),
                              float(pos_weight), _p(grad), _p(loss), _p(status), _stream(stream)))


def cnn_adam_step(params, params_bf16, m, v, grad, lr, beta1, beta2, eps, step, stream=None):
    _check(lib().cnn_adam_step(_p(params), _p(params_bf16), _p(m), _p(v), _p(grad), int(params.numel()),
                               float(lr), float(beta1), float(beta2), float(eps), int(step), _stream(stream)))
