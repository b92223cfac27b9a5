"""Batched workloads at full size, in the launch configuration the benchmark
times (autotuned detector tiles, the whole path replayed as one HIP graph),
compared with the per-image oracle on every pair; and the autotuner's own contract
(results never depend on the tiles it picks)."""
import os

import numpy as np
import pytest

import oracle
from synth import configs, scenes
from synth.configs import Params
from tests.parity_util import compare_kps, compare_matches, oracle_image, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fe_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_04090_amd import frontend
    return frontend


def snapshot(fe):
    outs = [fe.results(i) for i in range(fe.n)]
    m = [fe.matches(p) for p in range(fe.n // 2)]
    return outs, m


def assert_same(a, b):
    for ra, rb in zip(a[0], b[0]):
        assert ra.keys() == rb.keys()
        for k in ra:
            assert np.array_equal(ra[k], rb[k]), k
    for ma, mb in zip(a[1], b[1]):
        for x, y in zip(ma, mb):
            assert np.array_equal(x, y)


def test_autotune_keeps_results(fe_mod, pattern):
    import torch
    imgs = []
    for k, (w, h) in enumerate([(320, 240), (376, 240), (620, 188), (640, 360)]):
        l, r = scenes.stereo_pair(500 + k, w, h, 80, 40)
        imgs += [l, r]
    p = Params()
    fe = fe_mod.Frontend(p, [(im.shape[1], im.shape[0]) for im in imgs], pattern)
    try:
        fe.upload(imgs)
        fe.run()
        torch.cuda.synchronize()
        before = snapshot(fe)
        tw0, th0 = fe.tiles()
        assert tw0 == [128] * p.n_levels and th0 == [32] * p.n_levels
        rep = fe.autotune(reps=2)
        say("autotune report", rep)
        tw, th = fe.tiles()
        for l in range(p.n_levels):
            c = oracle.cell_size(p.cell0, l)
            assert rep["tile_w"][l] % c == 0 and rep["tile_h"][l] % c == 0
            assert c <= rep["tile_w"][l] <= max(128, c) and c <= rep["tile_h"][l] <= max(32, c)
            assert rep["n_tried"][l] >= 1 and rep["us"][l] > 0 and rep["us"][l] <= rep["us_before"][l]
            assert tw[l] // c == rep["tile_w"][l] // c and th[l] // c == rep["tile_h"][l] // c
        # the pyramid pass timed both schedules and installed the one it reports
        from paper_2410_04090_amd import vsfe
        pr = rep["pyramid"]
        assert pr["n_tried"] >= 3 and pr["us"] > 0 and pr["us_worst"] >= pr["us"]
        sched, ptw, pth = vsfe.batch_pyramid_get(fe.batch)
        assert pr["schedule"] == {vsfe.PYR_LEVELS: "levels", vsfe.PYR_TOWER: "tower"}[sched]
        if sched == vsfe.PYR_TOWER:
            assert [ptw, pth] == pr["tile"]
        fe.run()
        torch.cuda.synchronize()
        assert_same(before, snapshot(fe))
        # an explicit, very different shape per level gives the same bits too
        fe.set_tiles([16] * p.n_levels, [8] * p.n_levels)
        fe.run()
        torch.cuda.synchronize()
        assert_same(before, snapshot(fe))
        # and the oracle agrees with all of them
        for i in (0, 7):
            _, ref = oracle_image(imgs[i], p, pattern)
            compare_kps(ref, before[0][i], i)
    finally:
        fe.close()


def run_bench_config(fe_mod, wl, imgs, pattern):
    import torch
    fe = fe_mod.Frontend(wl.params, wl.image_sizes(), pattern)
    fe.upload(imgs)
    rep = fe.autotune(reps=2)
    say("tiles", rep["tile_w"], rep["tile_h"])
    fe.capture()
    fe.kp_count.zero_()
    fe.desc.zero_()
    torch.cuda.synchronize()
    fe.replay()
    torch.cuda.synchronize()
    assert int(fe.status.item()) == 0
    return fe


def oracle_refs(imgs, params, pattern, images, threads):
    """Oracle keypoints of the given images, `threads` images at a time (the
    C oracle keeps no state and runs with the interpreter lock released)."""
    oracle.lib()
    if threads <= 1:
        return {i: oracle_image(imgs[i], params, pattern)[1] for i in images}
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return dict(zip(images, ex.map(lambda i: oracle_image(imgs[i], params, pattern)[1], images)))


def check_pairs(fe, imgs, params, pattern, pairs, threads=1):
    pairs = list(pairs)
    refs = oracle_refs(imgs, params, pattern, [i for pr in pairs for i in (2 * pr, 2 * pr + 1)], threads)
    for pr in pairs:
        for i in (2 * pr, 2 * pr + 1):
            compare_kps(refs[i], fe.results(i), i)
        n = compare_matches(fe, pr, refs[2 * pr], refs[2 * pr + 1], params)
        say("pair", pr, imgs[2 * pr].shape, "keypoints", len(refs[2 * pr]["x"]), len(refs[2 * pr + 1]["x"]),
            "matches", n)


def check_invariants(fe, params):
    """Properties of every image of the batch (sizes the oracle is not run on)."""
    counts = fe.kp_count.cpu().numpy()
    assert (counts >= 0).all() and (counts <= params.n_max).all()
    for i in range(fe.n):
        r = fe.results(i)
        # canonical order: level, then cell row, then cell column (strictly increasing)
        key = [(int(lv), int(y) // oracle.cell_size(params.cell0, int(lv)), int(x) // oracle.cell_size(params.cell0, int(lv)))
               for lv, x, y in zip(r["level"], r["x"], r["y"])]
        assert all(a < b for a, b in zip(key, key[1:])), i
        assert (r["bin"] < 30).all()
    for pr in range(fe.n // 2):
        idx, dist, disp = fe.matches(pr)
        nr = int(counts[2 * pr + 1])
        ok = idx >= 0
        assert (idx[ok] < nr).all()
        assert (dist[ok] <= params.match_th).all() and (dist[~ok] == 0xFFFF).all()
        assert (disp[ok] >= 0).all() and (disp[ok] <= params.d_max).all() and (disp[~ok] == -1).all()


def test_mixed_batch_full_size(fe_mod, pattern):
    """32 pairs of four sizes (640x480, 752x480, 1241x376, 1280x720): every
    pair against the oracle."""
    wl = configs.batch32_mixed()
    say("case: mixed batch", wl.name)
    imgs = wl.images()
    fe = run_bench_config(fe_mod, wl, imgs, pattern)
    try:
        check_invariants(fe, wl.params)
        check_pairs(fe, imgs, wl.params, pattern, range(len(wl.sizes)))
    finally:
        fe.close()


def test_1080p_batch_full_size(fe_mod, pattern):
    """64 pairs of 1920x1080 with at most 4000 keypoints per image: every
    pair against the oracle (up to 16 oracle images at a time)."""
    wl = configs.batch64_1080p()
    say("case: 1080p batch", wl.name)
    imgs = wl.images()
    fe = run_bench_config(fe_mod, wl, imgs, pattern)
    try:
        check_invariants(fe, wl.params)
        check_pairs(fe, imgs, wl.params, pattern, range(len(wl.sizes)), threads=min(16, os.cpu_count() or 1))
        assert int(fe.kp_count.max().item()) == wl.params.n_max      # the cap is exercised
    finally:
        fe.close()
