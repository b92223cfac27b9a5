"""CPU oracle of the stereo front-end: test infrastructure only.

A ctypes front for ``liboracle.so`` (plain C in this directory) plus the
fp64 numpy oracle of the learned cell proposer (``cnn.py``).  Only the
tests, the smoke check and the benchmark's CPU-baseline leg use it; the GPU
library never loads it and shares no code with it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["pyramid.c", "fast.c", "detect.c", "orb.c", "stereo.c", "refine.c", "track.c", "frontend.c"]


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc -O2 (plain scalar C)."""
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-Wall", "-shared", "-fPIC",
           "-o", LIB_PATH] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


class OrParams(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "eps_hi", "eps_lo", "p_min", "p_max", "border", "n_levels", "cell0",
        "pfa", "nms_mode", "nms_radius", "n_max", "blur", "d_max", "match_th", "row_band")]


class OrKps(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("level", C.c_void_p),
                ("flags", C.c_void_p), ("score", C.c_void_p), ("x0", C.c_void_p),
                ("y0", C.c_void_p), ("kl", C.c_void_p), ("kr", C.c_void_p),
                ("bin", C.c_void_p), ("desc", C.c_void_p), ("capacity", C.c_int32)]


def _declare(L):
    i32, p = C.c_int32, C.c_void_p
    pi = C.POINTER(C.c_int32)
    L.or_level_size.argtypes = [i32, i32, i32, pi, pi]
    L.or_cell_size.argtypes = [i32, i32]
    L.or_cell_size.restype = i32
    L.or_scale_q16.argtypes = [i32]
    L.or_scale_q16.restype = C.c_int64
    L.or_project.argtypes = [i32, i32, i32]
    L.or_project.restype = i32
    L.or_pyramid_bytes.argtypes = [i32, i32, i32]
    L.or_pyramid_bytes.restype = C.c_int64
    L.or_pyramid.argtypes = [p, i32, i32, i32, i32, p]
    L.or_longest_run.argtypes = [p]
    L.or_longest_run.restype = i32
    L.or_mask_is_corner.argtypes = [C.c_uint32, i32, i32]
    L.or_mask_is_corner.restype = i32
    L.or_is_corner.argtypes = [p, i32, i32, i32, i32, i32, i32, pi, pi]
    L.or_is_corner.restype = i32
    L.or_score.argtypes = [p, i32, i32, i32]
    L.or_score.restype = i32
    L.or_crf.argtypes = [p, i32, i32, i32, i32, i32, i32, p]
    L.or_cull_level.argtypes = [p, i32, i32, i32, C.POINTER(OrParams), p, p]
    L.or_detect.argtypes = [p, i32, i32, C.POINTER(OrParams), p, C.POINTER(OrKps)]
    L.or_detect.restype = i32
    L.or_cell_runs.argtypes = [i32, i32, i32, i32, i32, i32, i32, p]
    L.or_cell_runs.restype = i32
    L.or_pfa_from_records.argtypes = [i32, p, p, p, p, i32, i32, i32, i32, i32, p, p, p]
    L.or_pfa_from_records.restype = i32
    L.or_blur_level.argtypes = [p, i32, i32, p]
    L.or_rot_table.argtypes = [p, p]
    L.or_bin_table.argtypes = [p, p]
    L.or_moments.argtypes = [p, i32, i32, i32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.or_angle_bin.argtypes = [C.c_int64, C.c_int64]
    L.or_angle_bin.restype = i32
    L.or_rotate_point.argtypes = [i32, i32, i32, pi, pi]
    L.or_describe.argtypes = [p, i32, i32, C.POINTER(OrParams), p, i32, C.POINTER(OrKps)]
    L.or_stereo.argtypes = [i32, C.POINTER(OrKps), i32, C.POINTER(OrKps), C.POINTER(OrParams),
                            p, p, p]
    L.or_stereo_refine.argtypes = [p, p, i32, i32, i32, C.POINTER(OrKps), C.POINTER(OrKps), p, i32, i32, p, p]
    L.or_feature_match.argtypes = [i32, C.POINTER(OrKps), i32, C.POINTER(OrKps), i32, i32, i32, i32, p, p, p]
    L.or_frontend_pair.argtypes = [p, p, i32, i32, C.POINTER(OrParams), p,
                                   C.POINTER(OrKps), pi, C.POINTER(OrKps), pi, p, p, p]
    L.or_frontend_pair.restype = i32


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def make_params(params) -> OrParams:
    """Accept a dataclass / dict with the front-end parameter names."""
    d = params if isinstance(params, dict) else params.as_dict()
    d = dict(d)
    d.setdefault("nms_radius", 1)
    return OrParams(**{k: int(d[k]) for k, _ in OrParams._fields_})


# ----------------------------------------------------------------- geometry
def level_size(W, H, l):
    a, b = C.c_int32(), C.c_int32()
    lib().or_level_size(W, H, l, C.byref(a), C.byref(b))
    return a.value, b.value


def cell_size(cell0, l):
    return lib().or_cell_size(cell0, l)


def scale_q16(l):
    return lib().or_scale_q16(l)


def project(x, l, W0):
    return lib().or_project(x, l, W0)


# ----------------------------------------------------------------- pyramid
def pyramid_packed(img: np.ndarray, L: int) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    out = np.zeros(lib().or_pyramid_bytes(W, H, L), dtype=np.uint8)
    lib().or_pyramid(_ptr(img), W, H, W, L, _ptr(out))
    return out


def split_levels(packed: np.ndarray, W: int, H: int, L: int):
    out, at = [], 0
    for l in range(L):
        w, h = level_size(W, H, l)
        out.append(packed[at:at + w * h].reshape(h, w))
        at += w * h
    return out


def pyramid(img: np.ndarray, L: int):
    H, W = img.shape
    return split_levels(pyramid_packed(img, L), W, H, L)


# ----------------------------------------------------------------- FAST / FC
def longest_run(labels) -> int:
    a = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
    assert a.shape == (16,)
    return lib().or_longest_run(_ptr(a))


def mask_is_corner(mask16: int, p_min=9, p_max=13) -> bool:
    return bool(lib().or_mask_is_corner(mask16, p_min, p_max))


def is_corner(lvl: np.ndarray, x, y, eps, p_min=9, p_max=13):
    lvl = np.ascontiguousarray(lvl, dtype=np.uint8)
    nb, nd = C.c_int32(), C.c_int32()
    r = lib().or_is_corner(_ptr(lvl), lvl.shape[1], x, y, eps, p_min, p_max,
                           C.byref(nb), C.byref(nd))
    return bool(r), nb.value, nd.value


def score(lvl: np.ndarray, x, y) -> int:
    lvl = np.ascontiguousarray(lvl, dtype=np.uint8)
    return lib().or_score(_ptr(lvl), lvl.shape[1], x, y)


def crf(lvl: np.ndarray, eps=20, p_min=9, p_max=13, border=3) -> np.ndarray:
    lvl = np.ascontiguousarray(lvl, dtype=np.uint8)
    H, W = lvl.shape
    out = np.zeros((H, W), dtype=np.uint16)
    lib().or_crf(_ptr(lvl), W, H, eps, p_min, p_max, border, _ptr(out))
    return out


def cull_level(lvl: np.ndarray, c: int, params):
    lvl = np.ascontiguousarray(lvl, dtype=np.uint8)
    H, W = lvl.shape
    ncx, ncy = (W + c - 1) // c, (H + c - 1) // c
    key = np.zeros((ncy, ncx), dtype=np.uint32)
    flag = np.zeros((ncy, ncx), dtype=np.uint8)
    pp = make_params(params)
    lib().or_cull_level(_ptr(lvl), W, H, c, C.byref(pp), _ptr(key), _ptr(flag))
    return key, flag


# ----------------------------------------------------------------- keypoints
KP_FIELDS = [("x", np.uint16), ("y", np.uint16), ("level", np.uint8), ("flags", np.uint8),
             ("score", np.uint16), ("x0", np.uint16), ("y0", np.uint16), ("kl", np.uint8),
             ("kr", np.uint32), ("bin", np.uint8)]


def _alloc_kps(cap: int, with_desc: bool = True):
    d = {k: np.zeros(cap, dtype=t) for k, t in KP_FIELDS}
    d["desc"] = np.zeros((cap, 8), dtype=np.uint32) if with_desc else None
    return d


def _kps_struct(d, cap):
    s = OrKps()
    for k, _ in KP_FIELDS:
        setattr(s, k, _ptr(d[k]))
    s.desc = _ptr(d["desc"]) if d.get("desc") is not None else None
    s.capacity = cap
    return s


def _trim(d, n):
    return {k: (v[:n] if v is not None else None) for k, v in d.items()}


def detect(packed_pyr: np.ndarray, W: int, H: int, params, cell_mask0=None):
    pp = make_params(params)
    cap = max(1, _total_cells(W, H, pp))
    d = _alloc_kps(cap)
    s = _kps_struct(d, cap)
    m = None
    if cell_mask0 is not None:
        cell_mask0 = np.ascontiguousarray(cell_mask0, dtype=np.uint8)
        m = _ptr(cell_mask0)
    n = lib().or_detect(_ptr(packed_pyr), W, H, C.byref(pp), m, C.byref(s))
    if n < 0:
        raise ValueError("oracle detect: invalid parameters")
    return _trim(d, n)


def _total_cells(W, H, pp):
    t = 0
    for l in range(pp.n_levels):
        w, h = level_size(W, H, l)
        c = cell_size(pp.cell0, l)
        t += ((w + c - 1) // c) * ((h + c - 1) // c)
    return t


def cell_runs(level, cx, cy, c, W0, H0, cell0, mask0) -> bool:
    """Learned gating footprint test of one level-l cell (mask0: level-0 cells)."""
    m = np.ascontiguousarray(mask0, dtype=np.uint8)
    return bool(lib().or_cell_runs(level, cx, cy, c, W0, H0, cell0, _ptr(m)))


def pfa_from_records(level, x0, y0, resp, W, H, n_levels, nms_mode=0, nms_radius=1):
    level = np.ascontiguousarray(level, dtype=np.int32)
    x0 = np.ascontiguousarray(x0, dtype=np.int32)
    y0 = np.ascontiguousarray(y0, dtype=np.int32)
    resp = np.ascontiguousarray(resp, dtype=np.int32)
    n = len(level)
    kl = np.zeros(max(n, 1), np.int32)
    kr = np.zeros(max(n, 1), np.int32)
    keep = np.zeros(max(n, 1), np.int32)
    rc = lib().or_pfa_from_records(n, _ptr(level), _ptr(x0), _ptr(y0), _ptr(resp), W, H,
                                   n_levels, nms_mode, nms_radius, _ptr(kl), _ptr(kr),
                                   _ptr(keep))
    if rc:
        raise ValueError("oracle pfa: rc=%d" % rc)
    return kl[:n], kr[:n], keep[:n].astype(bool)


# ----------------------------------------------------------------- ORB
def blur_level(lvl: np.ndarray) -> np.ndarray:
    lvl = np.ascontiguousarray(lvl, dtype=np.uint8)
    H, W = lvl.shape
    out = np.zeros_like(lvl)
    lib().or_blur_level(_ptr(lvl), W, H, _ptr(out))
    return out


def rot_table():
    c = np.zeros(30, np.int32)
    s = np.zeros(30, np.int32)
    lib().or_rot_table(_ptr(c), _ptr(s))
    return c, s


def bin_table():
    c = np.zeros(30, np.int32)
    s = np.zeros(30, np.int32)
    lib().or_bin_table(_ptr(c), _ptr(s))
    return c, s


def moments(lvl: np.ndarray, x, y):
    lvl = np.ascontiguousarray(lvl, dtype=np.uint8)
    a, b = C.c_int64(), C.c_int64()
    lib().or_moments(_ptr(lvl), lvl.shape[1], x, y, C.byref(a), C.byref(b))
    return a.value, b.value


def angle_bin(mx, my) -> int:
    return lib().or_angle_bin(int(mx), int(my))


def rotate_point(u, v, k):
    a, b = C.c_int32(), C.c_int32()
    lib().or_rotate_point(u, v, k, C.byref(a), C.byref(b))
    return a.value, b.value


def describe(packed_pyr: np.ndarray, W: int, H: int, params, pattern: np.ndarray, kps: dict):
    """Fill kps['bin'] and kps['desc'] in place (copies are made contiguous)."""
    pp = make_params(params)
    n = len(kps["x"])
    d = {k: np.ascontiguousarray(kps[k]).copy() for k, _ in KP_FIELDS}
    d["desc"] = np.zeros((max(n, 1), 8), dtype=np.uint32)
    for k, _ in KP_FIELDS:
        if len(d[k]) == 0:
            d[k] = np.zeros(1, dtype=d[k].dtype)
    s = _kps_struct(d, max(n, 1))
    pat = np.ascontiguousarray(pattern, dtype=np.int8)
    lib().or_describe(_ptr(packed_pyr), W, H, C.byref(pp), _ptr(pat), n, C.byref(s))
    out = dict(kps)
    out["bin"] = d["bin"][:n]
    out["desc"] = d["desc"][:n]
    return out


def stereo(kl: dict, kr: dict, params):
    pp = make_params(params)
    nl, nr = len(kl["x"]), len(kr["x"])

    def prep(k, n):
        d = {f: np.ascontiguousarray(k[f]) if n else np.zeros(1, dtype=t) for f, t in KP_FIELDS}
        d["desc"] = np.ascontiguousarray(k["desc"]) if n else np.zeros((1, 8), np.uint32)
        return d, _kps_struct(d, max(n, 1))

    dl, sl = prep(kl, nl)
    dr, sr = prep(kr, nr)
    idx = np.zeros(max(nl, 1), np.int32)
    dist = np.zeros(max(nl, 1), np.uint16)
    disp = np.zeros(max(nl, 1), np.int16)
    lib().or_stereo(nl, C.byref(sl), nr, C.byref(sr), C.byref(pp), _ptr(idx), _ptr(dist),
                    _ptr(disp))
    return idx[:nl], dist[:nl], disp[:nl]


def stereo_refine(pyr_l: np.ndarray, pyr_r: np.ndarray, W: int, H: int, kl: dict, kr: dict, idx,
                  half_window=5, search_radius=5):
    """Sub-pixel disparities (1/256 pixel, native scale; INT32_MIN = not
    refined) and least SADs of the matches idx of a pair (packed pyramids)."""
    nl, nr = len(kl["x"]), len(kr["x"])

    def prep(k, n):
        d = {f: np.ascontiguousarray(k[f]) if n else np.zeros(1, dtype=t) for f, t in KP_FIELDS}
        d["desc"] = None
        return d, _kps_struct(d, max(n, 1))

    dl, sl = prep(kl, nl)
    dr, sr = prep(kr, nr)
    ix = np.ascontiguousarray(idx, dtype=np.int32) if nl else np.full(1, -1, np.int32)
    disp = np.zeros(max(nl, 1), np.int32)
    sad = np.zeros(max(nl, 1), np.uint32)
    lib().or_stereo_refine(_ptr(np.ascontiguousarray(pyr_l, dtype=np.uint8)),
                           _ptr(np.ascontiguousarray(pyr_r, dtype=np.uint8)), W, H, nl, C.byref(sl), C.byref(sr),
                           _ptr(ix), half_window, search_radius, _ptr(disp), _ptr(sad))
    return disp[:nl], sad[:nl]


def feature_match(kq: dict, kr: dict, radius, level_band, match_th, ratio_pct):
    """Matches of query keypoints kq against reference keypoints kr (dicts
    with x0, y0, level, desc): (idx, best distance, runner-up distance)."""
    nq, nr = len(kq["x0"]), len(kr["x0"])

    def prep(k, n):
        d = {}
        for f, t in KP_FIELDS:
            a = np.asarray(k[f], dtype=t) if (f in k and n) else np.zeros(max(n, 1), dtype=t)
            d[f] = np.ascontiguousarray(a)
        d["desc"] = np.ascontiguousarray(k["desc"], dtype=np.uint32) if n else np.zeros((1, 8), np.uint32)
        return d, _kps_struct(d, max(n, 1))

    dq, sq = prep(kq, nq)
    dr, sr = prep(kr, nr)
    idx = np.zeros(max(nq, 1), np.int32)
    d1 = np.zeros(max(nq, 1), np.uint16)
    d2 = np.zeros(max(nq, 1), np.uint16)
    lib().or_feature_match(nq, C.byref(sq), nr, C.byref(sr), radius, level_band, match_th, ratio_pct, _ptr(idx),
                           _ptr(d1), _ptr(d2))
    return idx[:nq], d1[:nq], d2[:nq]


def frontend_image(img: np.ndarray, params, pattern=None, cell_mask0=None):
    """Pyramid + detection (+ description when ``pattern`` is given)."""
    pp = make_params(params)
    H, W = img.shape
    packed = pyramid_packed(img, pp.n_levels)
    kps = detect(packed, W, H, params, cell_mask0)
    if pattern is not None:
        kps = describe(packed, W, H, params, pattern, kps)
    return packed, kps


def frontend_pair(left: np.ndarray, right: np.ndarray, params, pattern, cell_mask0=None):
    _, kl = frontend_image(left, params, pattern, cell_mask0)
    _, kr = frontend_image(right, params, pattern, cell_mask0)
    idx, dist, disp = stereo(kl, kr, params)
    return kl, kr, (idx, dist, disp)


def frontend_pair_native(left: np.ndarray, right: np.ndarray, params, pattern):
    """The same pipeline in one C call (used to time the oracle)."""
    pp = make_params(params)
    H, W = left.shape
    cap = max(1, _total_cells(W, H, pp))
    dl, dr = _alloc_kps(cap), _alloc_kps(cap)
    sl, sr = _kps_struct(dl, cap), _kps_struct(dr, cap)
    nl, nr = C.c_int32(), C.c_int32()
    idx = np.zeros(cap, np.int32)
    dist = np.zeros(cap, np.uint16)
    disp = np.zeros(cap, np.int16)
    L = np.ascontiguousarray(left, dtype=np.uint8)
    R = np.ascontiguousarray(right, dtype=np.uint8)
    pat = np.ascontiguousarray(pattern, dtype=np.int8)
    rc = lib().or_frontend_pair(_ptr(L), _ptr(R), W, H, C.byref(pp), _ptr(pat), C.byref(sl),
                                C.byref(nl), C.byref(sr), C.byref(nr), _ptr(idx), _ptr(dist),
                                _ptr(disp))
    if rc:
        raise ValueError("oracle frontend_pair failed")
    return (_trim(dl, nl.value), _trim(dr, nr.value),
            (idx[:nl.value], dist[:nl.value], disp[:nl.value]))
