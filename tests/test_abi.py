"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/vsfe.h, and its host-only calls validate arguments
(no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2410_04090_amd import vsfe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vsfe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z0-9_]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "pyramid_build" in names and "stereo_match" in names and len(names) >= 17
    lib = vsfe.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_exports():
    for n in declared_functions():
        assert n in vsfe.EXPORTS, n


def test_params_validation():
    p = vsfe.make_params()
    assert vsfe.params_check(p) == 0
    for field, bad in [("eps_hi", 300), ("eps_lo", 30), ("p_min", 0), ("p_max", 17), ("border", 2),
                       ("n_levels", 13), ("cell0", 40), ("nms_radius", 4), ("n_max", 0), ("row_band", 5),
                       ("match_th", 257), ("pfa", 2)]:
        q = vsfe.make_params(**{field: bad})
        assert vsfe.params_check(q) == vsfe.EINVAL, field
        assert vsfe.lib().vsfe_last_error().decode()
    # p_min > p_max
    assert vsfe.params_check(vsfe.make_params(p_min=12, p_max=10)) == vsfe.EINVAL
    # smallest cells at the deepest level stay >= 1 pixel
    assert vsfe.params_check(vsfe.make_params(cell0=8, n_levels=12)) == 0
    assert vsfe.level_geometry(vsfe.make_params(cell0=8), 4000, 4000, 11)[2] == 1


def test_level_geometry():
    p = vsfe.make_params()
    assert vsfe.level_geometry(p, 1241, 376, 0) == (1241, 376, 32)
    assert vsfe.level_geometry(p, 1241, 376, 7) == (346, 105, 8)
    with pytest.raises(vsfe.VsfeError):
        vsfe.level_geometry(p, 0, 10, 0)


def test_batch_plan_sizes():
    p = vsfe.make_params()
    info = vsfe.batch_plan(p, [1241, 1241], [376, 376], [1280, 1280], [0, 1280 * 376])
    assert info.n_cells == 2 * 4216          # cells per 1241x376 image over 8 levels
    assert info.n_cells0 == 2 * 39 * 12
    assert info.kp_capacity == 2 * 2000 and info.match_capacity == 2000
    assert info.input_bytes == 2 * 1280 * 376
    assert info.crf_elems == 2 * 1444097     # pixels of all levels
    with pytest.raises(vsfe.VsfeError):
        vsfe.batch_plan(p, [100], [100], [50], [0])      # pitch < width
    with pytest.raises(vsfe.VsfeError):
        vsfe.batch_plan(p, [1], [1], [1], [0])           # level 1 would be empty


def test_ctx_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import numpy as np
    p = vsfe.make_params()
    with pytest.raises(vsfe.VsfeError) as e:
        vsfe.ctx_create(p, np.zeros((256, 4), np.int8))
    assert e.value.code in (vsfe.EUNSUPPORTED, vsfe.EHIP)


def test_pattern_outside_disc_rejected():
    import numpy as np
    p = vsfe.make_params()
    pat = np.zeros((256, 4), np.int8)
    pat[3] = (15, 15, 0, 0)
    with pytest.raises(vsfe.VsfeError) as e:
        vsfe.ctx_create(p, pat)
    assert e.value.code == vsfe.EINVAL


def test_autotune_and_tiles_reject_null_arguments():
    lib = vsfe.lib()
    rep = vsfe.TuneReport()
    w = (C.c_int32 * vsfe.MAX_LEVELS)(*([64] * vsfe.MAX_LEVELS))
    assert lib.vsfe_batch_autotune(None, None, None, None, None, None, 3, None, C.byref(rep)) == vsfe.EINVAL
    assert lib.vsfe_batch_set_tiles(None, w, w) == vsfe.EINVAL
    assert lib.vsfe_batch_tiles_get(None, w, w) == vsfe.EINVAL
    assert b"null" in lib.vsfe_last_error()


def test_detect_levels_rejects_null_arguments():
    lib = vsfe.lib()
    assert lib.fast_br_detect_levels(None, None, None, None, None, None, 0, 1, None, None) == vsfe.EINVAL
    assert b"null" in lib.vsfe_last_error()


def test_batch_plan_refuses_proposer_overflow():
    """A batch within the image count and size limits whose proposer tables
    (32-bit prefix sums of conv1 pixels over the batch) would overflow is
    refused at planning time with ECAPACITY, before anything is allocated."""
    p = vsfe.make_params()
    n, side = 400, 8192                       # 400 x 2371^2 conv1 pixels > 2^31
    with pytest.raises(vsfe.VsfeError) as e:
        vsfe.batch_plan(p, [side] * n, [side] * n, [side] * n, [i * side * side for i in range(n)])
    assert e.value.code == vsfe.ECAPACITY
    # the same images with 3 levels (no proposer) plan fine
    info = vsfe.batch_plan(vsfe.make_params(n_levels=3), [side] * 2, [side] * 2, [side] * 2, [0, side * side])
    assert info.n_images == 2


def test_probe_argument_checks():
    """The ceiling probes reject unknown kinds, sizes out of range and null
    buffers on the host, before any launch."""
    L = vsfe.lib()
    dummy = C.c_void_p(16)
    for kind, blocks, iters, sink, clocks in ((0, 1, 1, dummy, dummy), (3, 1, 1, dummy, dummy),
                                              (vsfe.PROBE_VALU, 0, 1, dummy, dummy),
                                              (vsfe.PROBE_LDS, 1, 0, dummy, dummy),
                                              (vsfe.PROBE_VALU, 1 << 21, 1, dummy, dummy),
                                              (vsfe.PROBE_LDS, 1 << 14, 1 << 13, dummy, dummy),
                                              (vsfe.PROBE_VALU, 1, 1, None, dummy),
                                              (vsfe.PROBE_LDS, 1, 1, dummy, None)):
        assert L.vsfe_probe(kind, blocks, iters, sink, clocks, None) == vsfe.EINVAL
