"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Every stage is compared element by element on seeded inputs: pyramid
levels, per-cell keys (with the fallback flag), the response dump, the
aggregated keypoint lists, orientation bins, descriptors and matches.
"""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from synth import configs, scenes
from synth.configs import Params
from tests.parity_util import (compare_cells, compare_crf, compare_kps, compare_matches,
                               compare_pyramid, oracle_image, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fe_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_04090_amd import frontend
    return frontend


def run_and_compare(fe_mod, imgs, params, pattern, full_stages=True, tile=None, mask=None, describe=True,
                    overlap=None, schedule=None, layout=None):
    sizes = [(im.shape[1], im.shape[0]) for im in imgs]
    say("case: sizes=%s params=%s tile=%s mask=%s schedule=%s layout=%s" % (sizes[:4], params, tile,
                                                                            mask is not None, schedule, layout))
    fe = fe_mod.Frontend(params, sizes, pattern, tile=tile, with_crf=full_stages,
                         with_mask=mask is not None, layout=layout)
    try:
        if schedule is not None:
            from paper_2410_04090_amd import vsfe
            vsfe.batch_set_pyramid(fe.batch, schedule)
        fe.upload(imgs)
        mt = None
        if mask is not None:
            import torch
            fe.cell_mask.copy_(torch.from_numpy(np.concatenate([m.reshape(-1) for m in mask])))
            mt = fe.cell_mask
        fe.run(mask=mt, describe=describe and params.border >= 15, overlap=overlap)
        import torch
        torch.cuda.synchronize()
        assert int(fe.status.item()) == 0
        refs = []
        for i, img in enumerate(imgs):
            if full_stages:
                levels = compare_pyramid(fe, i, img, params)
                if mask is None:
                    compare_cells(fe, i, levels, params)
                compare_crf(fe, i, levels, params)
            _, ref = oracle_image(img, params, pattern, None if mask is None else mask[i])
            got = fe.results(i)
            compare_kps(ref, got, i, describe=describe and params.border >= 15)
            refs.append(ref)
        n_acc = 0
        if describe and params.border >= 15 and fe.stereo:
            for pr in range(len(imgs) // 2):
                n_acc += compare_matches(fe, pr, refs[2 * pr], refs[2 * pr + 1], params)
        return fe, refs, n_acc
    finally:
        fe.close()


def test_mono_752x480(fe_mod, pattern):
    w = configs.mono_752x480()
    imgs = w.images()
    _, refs, _ = run_and_compare(fe_mod, imgs, w.params, pattern, describe=False)
    assert len(refs[0]["x"]) > 100


def test_pair_1241x376(fe_mod, pattern):
    w = configs.pair_1241x376()
    _, refs, n_acc = run_and_compare(fe_mod, w.images(), w.params, pattern)
    assert len(refs[0]["x"]) > 500 and n_acc > 100


@pytest.mark.parametrize("seed", [3, 4])
def test_random_dense_pairs_with_cap(fe_mod, pattern, seed):
    """Uniform noise: a corner in almost every cell, so the cap binds."""
    a = scenes.random_image(seed, 257, 193)
    b = scenes.random_image(seed + 100, 257, 193)
    p = Params(n_max=150)
    _, refs, _ = run_and_compare(fe_mod, [a, b], p, pattern)
    assert len(refs[0]["x"]) == 150


def test_more_keypoints_than_the_slot_map(fe_mod, pattern):
    """Over 8192 keypoints per image (small cells, no PFA, no binding cap):
    the aggregation writes them out cell by cell instead of slot by slot."""
    l, r = scenes.stereo_pair(5, 1280, 960, 600, 64)
    p = Params(cell0=16, pfa=0, n_max=65535)
    _, refs, _ = run_and_compare(fe_mod, [l, r], p, pattern, full_stages=False)
    assert min(len(ref["x"]) for ref in refs) > 8192


@pytest.mark.parametrize("W,H", [(97, 61), (130, 77), (33, 33), (640, 17)])
def test_ragged_and_tiny_sizes(fe_mod, pattern, W, H):
    """Odd sizes, partial cells, and levels narrower than twice the border."""
    l, r = scenes.stereo_pair(50 + W, W, H, 30, 10)
    run_and_compare(fe_mod, [l, r], Params(), pattern)


@pytest.mark.parametrize("W,H", [(8192, 160), (160, 8192)])
def test_maximum_side(fe_mod, pattern, W, H):
    """Images at the largest supported side (8192): 16-bit coordinates,
    projections and cell reciprocals at their range limits."""
    l, r = scenes.stereo_pair(77 + W, W, H, 300, 64)
    run_and_compare(fe_mod, [l, r], Params(), pattern, full_stages=False)


@pytest.mark.parametrize("W,H", [(97, 61), (640, 17), (1241, 376)])
@pytest.mark.parametrize("schedule", [1, 2])
def test_overlapped_path_sizes(fe_mod, pattern, W, H, schedule):
    """The overlapped run (level-0 detection on a second stream beside the
    pyramid build, the default for large batches; with one pyramid launch
    per level also levels 1..3 there, beside the later levels) against the
    oracle, down to levels with no cell, under both pyramid schedules."""
    l, r = scenes.stereo_pair(90 + W, W, H, 40, 12)
    run_and_compare(fe_mod, [l, r], Params(), pattern, full_stages=False, overlap=True, schedule=schedule)


def test_flat_images_no_keypoints(fe_mod, pattern):
    img = np.full((120, 160), 128, np.uint8)
    _, refs, _ = run_and_compare(fe_mod, [img, img.copy()], Params(), pattern)
    assert len(refs[0]["x"]) == 0


@pytest.mark.parametrize("variant", [
    dict(nms_mode=1), dict(nms_radius=0), dict(nms_radius=2), dict(nms_radius=3),
    dict(p_max=16, eps_lo=-1), dict(pfa=0, n_max=5000), dict(blur=0), dict(eps_hi=35, eps_lo=12),
    dict(cell0=16, n_levels=6), dict(p_min=12, p_max=14), dict(row_band=0, d_max=40, match_th=90),
    dict(n_levels=1), dict(n_levels=2), dict(n_levels=3),
])
def test_parameter_variants(fe_mod, pattern, variant):
    l, r = scenes.stereo_pair(77, 420, 260, 90, 40)
    p = replace(Params(), **variant)
    run_and_compare(fe_mod, [l, r], p, pattern)


@pytest.mark.parametrize("tile", [(8, 8), (32, 16), (128, 32), (96, 24), (64, 32)])
def test_tile_shapes_identical(fe_mod, pattern, tile):
    l, r = scenes.stereo_pair(78, 333, 201, 80, 40)
    run_and_compare(fe_mod, [l, r], Params(), pattern, tile=tile)


def test_mixed_batch(fe_mod, pattern):
    """Pairs of four sizes in one batch (the mixed-resolution workload at
    reduced scale)."""
    imgs = []
    for k, (w, h) in enumerate([(320, 240), (376, 240), (620, 188), (640, 360)]):
        l, r = scenes.stereo_pair(300 + k, w, h, 80, 40)
        imgs += [l, r]
    run_and_compare(fe_mod, imgs, Params(), pattern)


def test_gated_detection_matches_oracle(fe_mod, pattern):
    """Learned gating: a random level-0 cell mask applied on both sides."""
    l, r = scenes.stereo_pair(91, 400, 300, 100, 40)
    p = Params()
    rng = np.random.default_rng(5)
    ncx, ncy = (400 + 31) // 32, (300 + 31) // 32
    masks = [(rng.random((ncy, ncx)) < 0.4).astype(np.uint8) for _ in range(2)]
    run_and_compare(fe_mod, [l, r], p, pattern, full_stages=False, mask=masks)


@pytest.mark.parametrize("kind", ["zeros", "ones", "checker", "single", "rows"])
def test_gated_work_list_masks(fe_mod, pattern, kind):
    """The gated launch visits only tiles with a running cell (device-built
    work list); skipped cells must read as empty even after an ungated run
    left keys in them, for masks from none to all and structured ones."""
    import torch
    l, r = scenes.stereo_pair(95, 640, 360, 120, 40)
    p = Params()
    ncx, ncy = 640 // 32, (360 + 31) // 32
    m = np.zeros((ncy, ncx), np.uint8)
    if kind == "ones":
        m[:] = 1
    elif kind == "checker":
        m[(np.arange(ncy)[:, None] + np.arange(ncx)[None, :]) % 2 == 0] = 1
    elif kind == "single":
        m[ncy // 2, ncx // 2] = 1
    elif kind == "rows":
        m[::3, :] = 1
    say("case: gated work list, mask %s (%d of %d cells)" % (kind, int(m.sum()), m.size))
    fe = fe_mod.Frontend(p, [(640, 360)] * 2, pattern, with_mask=True)
    try:
        fe.upload([l, r])
        fe.run()                                       # ungated: keys in every cell
        fe.cell_mask.copy_(torch.from_numpy(np.concatenate([m.reshape(-1), m.reshape(-1)])))
        fe.run(mask=fe.cell_mask)
        torch.cuda.synchronize()
        assert int(fe.status.item()) == 0
        refs = []
        for i, img in enumerate((l, r)):
            _, ref = oracle_image(img, p, pattern, m)
            compare_kps(ref, fe.results(i), i)
            refs.append(ref)
            if kind == "zeros":
                assert len(ref["x"]) == 0
                for lv in range(p.n_levels):
                    assert not fe.cell_keys_level(i, lv).any()
        compare_matches(fe, 0, refs[0], refs[1], p)
    finally:
        fe.close()


def test_deterministic_repeats(fe_mod, pattern):
    import torch
    w = configs.pair_1241x376()
    imgs = w.images()
    fe = fe_mod.Frontend(w.params, [(1241, 376)] * 2, pattern)
    try:
        fe.upload(imgs)
        outs = []
        for _ in range(3):
            fe.run()
            torch.cuda.synchronize()
            outs.append([fe.results(0)["desc"].copy(), fe.matches(0)[0].copy()])
        for o in outs[1:]:
            assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
    finally:
        fe.close()


@pytest.mark.parametrize("overlap", [False, True])
def test_graph_replay_matches_eager(fe_mod, pattern, overlap):
    import torch
    w = configs.pair_1241x376()
    imgs = w.images()
    fe = fe_mod.Frontend(w.params, [(1241, 376)] * 2, pattern)
    try:
        fe.upload(imgs)
        fe.run(overlap=overlap)
        torch.cuda.synchronize()
        eager = (fe.results(0), fe.results(1), fe.matches(0))
        fe.capture(overlap=overlap)
        for rep in range(3):
            fe.kp_count.zero_()
            fe.desc.zero_()
            torch.cuda.synchronize()
            fe.replay()
            torch.cuda.synchronize()
            got = (fe.results(0), fe.results(1), fe.matches(0))
            for a, b in zip(eager[:2], got[:2]):
                for k in a:
                    assert np.array_equal(a[k], b[k]), (rep, k)
            for a, b in zip(eager[2], got[2]):
                assert np.array_equal(a, b)
    finally:
        fe.close()


def test_level_ranges_match_full_detection(fe_mod, pattern):
    """fast_br_detect_levels over disjoint level ranges, two of them running
    concurrently on different streams, writes exactly the cell keys of the
    full call; empty or out-of-range ranges are rejected."""
    import torch
    from paper_2410_04090_amd import vsfe
    imgs = []
    for k, (w, h) in enumerate([(640, 360), (333, 201)]):
        imgs += list(scenes.stereo_pair(700 + k, w, h, 100, 30))
    p = Params()
    fe = fe_mod.Frontend(p, [(im.shape[1], im.shape[0]) for im in imgs], pattern)
    try:
        fe.upload(imgs)
        c, b, L = fe.ctx, fe.batch, p.n_levels
        vsfe.pyramid_build(c, b, fe.images, fe.pyr, fe.status)
        vsfe.fast_br_detect(c, b, fe.images, fe.pyr, None, fe.cell_keys, None, fe.status)
        torch.cuda.synchronize()
        full = fe.cell_keys.cpu().numpy().copy()
        for cut in (1, 3):
            fe.cell_keys.fill_(-1)
            main = torch.cuda.current_stream()
            side = torch.cuda.Stream()
            side.wait_stream(main)
            vsfe.fast_br_detect_levels(c, b, fe.images, fe.pyr, None, fe.cell_keys, 0, cut, fe.status, side)
            vsfe.fast_br_detect_levels(c, b, fe.images, fe.pyr, None, fe.cell_keys, cut, L, fe.status, main)
            main.wait_stream(side)
            torch.cuda.synchronize()
            assert np.array_equal(fe.cell_keys.cpu().numpy(), full), cut
        assert int(fe.status.item()) == 0
        for lo, hi in ((2, 2), (-1, 1), (0, L + 1), (3, 1)):
            with pytest.raises(vsfe.VsfeError):
                vsfe.fast_br_detect_levels(c, b, fe.images, fe.pyr, None, fe.cell_keys, lo, hi, fe.status)
    finally:
        fe.close()


@pytest.mark.parametrize("sizes,levels", [
    ([(1241, 376), (1241, 376)], 8),
    ([(97, 61), (640, 17), (33, 33), (1920, 1080), (257, 193), (17, 9)], 8),
    ([(8192, 160), (160, 8192)], 8),
    ([(130, 77), (97, 61), (17, 9)], 12),
])
def test_pyramid_schedules(fe_mod, pattern, sizes, levels):
    """Both pyramid schedules (one launch per level; one launch for all
    levels with per-block halos) and several single-launch tiles write
    every level of every image exactly as the oracle builds it; pixels the
    schedule must not touch (row padding) keep their poison value."""
    import torch
    from paper_2410_04090_amd import vsfe
    p = Params(n_levels=levels)
    imgs = [scenes.random_image(900 + k, w, h) for k, (w, h) in enumerate(sizes)]
    fe = fe_mod.Frontend(p, sizes, pattern)
    try:
        fe.upload(imgs)
        cases = [(vsfe.PYR_LEVELS, 0, 0), (vsfe.PYR_TOWER, 0, 0), (vsfe.PYR_TOWER, 16, 4),
                 (vsfe.PYR_TOWER, 48, 8), (vsfe.PYR_TOWER, 128, 32), (vsfe.PYR_TOWER, 240, 4)]
        for sched, tw, th in cases:
            say("case: sizes=%s L=%d schedule=%d tile=%dx%d" % (sizes, levels, sched, tw, th))
            try:
                vsfe.batch_set_pyramid(fe.batch, sched, tw, th)
            except vsfe.VsfeError as e:
                # only a single-launch tile whose block does not fit may be refused
                assert sched == vsfe.PYR_TOWER and e.code == vsfe.ECAPACITY, e
                continue
            got = vsfe.batch_pyramid_get(fe.batch)
            assert got[0] == sched
            fe.pyr.fill_(0xA5)
            vsfe.pyramid_build(fe.ctx, fe.batch, fe.images, fe.pyr, fe.status)
            torch.cuda.synchronize()
            assert int(fe.status.item()) == 0
            for i, img in enumerate(imgs):
                compare_pyramid(fe, i, img, p)
                for l in range(1, levels):
                    li = fe.level_info(i, l)
                    if li.pitch > li.width:
                        pad = fe.pyr[li.offset:li.offset + li.pitch * li.height].cpu().numpy()
                        pad = pad.reshape(li.height, li.pitch)[:, li.width:]
                        assert (pad == 0xA5).all(), (i, l)
        vsfe.batch_set_pyramid(fe.batch, vsfe.PYR_AUTO)
    finally:
        fe.close()


def test_pyramid_schedule_errors(fe_mod, pattern):
    """Unknown schedules and tiles out of range are refused; a refused tile
    leaves the batch working."""
    from paper_2410_04090_amd import vsfe
    fe = fe_mod.Frontend(Params(), [(400, 256)], pattern)
    try:
        before = vsfe.batch_pyramid_get(fe.batch)
        # a single small image: the single-launch schedule with the small-batch tile
        assert before == (vsfe.PYR_TOWER, 64, 16)
        for sched, tw, th in ((3, 0, 0), (-1, 0, 0), (vsfe.PYR_TOWER, 18, 8), (vsfe.PYR_TOWER, 12, 8),
                              (vsfe.PYR_TOWER, 244, 8), (vsfe.PYR_TOWER, 64, 3), (vsfe.PYR_TOWER, 64, 65)):
            with pytest.raises(vsfe.VsfeError) as ei:
                vsfe.batch_set_pyramid(fe.batch, sched, tw, th)
            assert ei.value.code == vsfe.EINVAL
        assert vsfe.batch_pyramid_get(fe.batch) == before
        # explicit default tile (0 x 0) and back to the automatic choice
        vsfe.batch_set_pyramid(fe.batch, vsfe.PYR_LEVELS)
        assert vsfe.batch_pyramid_get(fe.batch) == (vsfe.PYR_LEVELS, 64, 16)
        vsfe.batch_set_pyramid(fe.batch, vsfe.PYR_AUTO)
        assert vsfe.batch_pyramid_get(fe.batch) == before
    finally:
        fe.close()


@pytest.mark.parametrize("align", [1, 4])
@pytest.mark.parametrize("schedule", [1, 2])
def test_unaligned_input_layout(fe_mod, pattern, align, schedule):
    """Input rows that are not 16-byte aligned (every level-0 read takes its
    byte-load path): odd pitches and offsets (align 1), and 4-byte aligned
    ones that are not 16-byte aligned (align 4: ORB and refinement read
    dwords, pyramid and detector bytes), under both pyramid schedules."""
    sizes = [(401, 257), (401, 257), (130, 77), (130, 77)]
    imgs = []
    for k in range(0, len(sizes), 2):
        w, h = sizes[k]
        imgs += list(scenes.stereo_pair(600 + k, w, h, 60, 20))
    pitches, offsets, at = [], [], align
    for (w, h) in sizes:
        pt = w + (3 if align == 1 else 4 + (-w) % 4)
        pitches.append(pt)
        offsets.append(at)
        at += pt * h + (5 if align == 1 else 4)
        if align == 4 and at % 16 == 0:
            at += 4
    assert any(o % 16 for o in offsets) and any(pt % 16 for pt in pitches)
    run_and_compare(fe_mod, imgs, Params(), pattern, layout=(pitches, offsets), schedule=schedule)


@pytest.mark.parametrize("schedule", [1, 2])
def test_pyramid_level_ranges(fe_mod, pattern, schedule):
    """pyramid_build_levels (one launch per level whatever the batch's
    schedule) over split ranges, the later range on a second stream after
    the first, builds the oracle's levels; ranges out of bounds are
    refused."""
    import torch
    from paper_2410_04090_amd import vsfe
    sizes = [(640, 360), (640, 360), (333, 201), (333, 201)]
    imgs = [scenes.random_image(950 + k, w, h) for k, (w, h) in enumerate(sizes)]
    p = Params()
    fe = fe_mod.Frontend(p, sizes, pattern)
    try:
        vsfe.batch_set_pyramid(fe.batch, schedule)
        fe.upload(imgs)
        L = p.n_levels
        for cut in (2, 4, 7):
            say("case: schedule=%d ranges [1, %d) [%d, %d)" % (schedule, cut, cut, L))
            fe.pyr.fill_(0)
            main = torch.cuda.current_stream()
            vsfe.pyramid_build_levels(fe.ctx, fe.batch, fe.images, fe.pyr, 1, cut, fe.status, main)
            side = torch.cuda.Stream()
            side.wait_stream(main)
            vsfe.pyramid_build_levels(fe.ctx, fe.batch, fe.images, fe.pyr, cut, L, fe.status, side)
            main.wait_stream(side)
            torch.cuda.synchronize()
            for i, img in enumerate(imgs):
                compare_pyramid(fe, i, img, p)
        for lo, hi in ((0, 2), (2, 2), (3, 1), (1, L + 1)):
            with pytest.raises(vsfe.VsfeError):
                vsfe.pyramid_build_levels(fe.ctx, fe.batch, fe.images, fe.pyr, lo, hi, fe.status)
        assert int(fe.status.item()) == 0
    finally:
        fe.close()
