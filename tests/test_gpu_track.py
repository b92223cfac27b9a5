"""Bit-exact parity of feature_match (through the C ABI) with the oracle's
descriptor matching: a frame's keypoints against the previous frame's
(here: the left views as the previous frame and the right views, whose
polygons moved by their disparities, as the current one), over radius,
level-band, threshold and ratio settings, on mixed and ragged sizes; and
against "map points" whose predicted positions were moved by up to 6
pixels, some far past the image (bucketed at the grid's edge)."""
import numpy as np
import pytest

import oracle
from synth import pattern as pat
from synth import scenes
from synth.configs import Params
from tests.parity_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def frames(pairs, params):
    from paper_2410_04090_amd.frontend import Frontend
    prev = [p[0] for p in pairs]
    cur = [p[1] for p in pairs]
    sizes = [(im.shape[1], im.shape[0]) for im in prev]
    fp = Frontend(params, sizes, pat.brief_pattern())
    fc = Frontend(params, sizes, pat.brief_pattern())
    fp.upload(prev)
    fc.upload(cur)
    fp.run(stereo=False)
    fc.run(stereo=False)
    return fp, fc


def gpu_match(torch, fc, fp, ref_kps, settings):
    from paper_2410_04090_amd import vsfe
    ws = torch.zeros(max(vsfe.feature_match_workspace(fc.batch), 4), dtype=torch.uint8, device="cuda")
    cap = int(fc.info.kp_capacity)
    idx = torch.zeros(cap, dtype=torch.int32, device="cuda")
    d1 = torch.zeros(cap, dtype=torch.int16, device="cuda")
    d2 = torch.zeros(cap, dtype=torch.int16, device="cuda")
    vsfe.feature_match(fc.ctx, fc.batch, fc.kps, fc.kp_count, fc.desc, ref_kps, fp.kp_count, fp.desc, *settings,
                       ws, idx, d1, d2, fc.status)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), d1.cpu().numpy().view(np.uint16), d2.cpu().numpy().view(np.uint16)


def check(torch, fc, fp, ref_kps, ref_lists, settings):
    idx, d1, d2 = gpu_match(torch, fc, fp, ref_kps, settings)
    n_max = fc.params.n_max
    n_acc = 0
    for i in range(fc.n):
        kq = fc.results(i)
        ri, r1, r2 = oracle.feature_match(kq, ref_lists[i], *settings)
        s = slice(i * n_max, i * n_max + len(kq["x"]))
        assert np.array_equal(ri, idx[s]), (i, settings, int(np.argmax(ri != idx[s])))
        assert np.array_equal(r1, d1[s]) and np.array_equal(r2, d2[s]), (i, settings)
        n_acc += int((ri >= 0).sum())
    return n_acc


SETTINGS = [(16, 1, 64, 90), (48, 2, 256, 0), (0, 0, 256, 100), (8, 0, 40, 75)]


def test_frame_to_frame(torch_mod):
    pairs = [scenes.stereo_pair(9001, 1241, 376, 200, 24), scenes.stereo_pair(9002, 640, 480, 150, 24),
             scenes.stereo_pair(9003, 333, 201, 60, 12), scenes.stereo_pair(9004, 97, 61, 10, 4)]
    fp, fc = frames(pairs, Params())
    try:
        refs = [fp.results(i) for i in range(fp.n)]
        for st in SETTINGS:
            say("case: feature_match frame to frame", st)
            n = check(torch_mod, fc, fp, fp.kps, refs, st)
            if st[0] >= 16:
                assert n > 100
    finally:
        fp.close()
        fc.close()


def test_map_points_with_predicted_positions(torch_mod):
    torch = torch_mod
    pairs = [scenes.stereo_pair(9011, 752, 480, 150, 16), scenes.stereo_pair(9012, 752, 480, 150, 16)]
    fp, fc = frames(pairs, Params())
    try:
        rng = np.random.default_rng(9)
        kps = {k: v.clone() for k, v in fp.kps.items()}
        x0 = kps["x0"].cpu().numpy().view(np.uint16).astype(np.int64)
        y0 = kps["y0"].cpu().numpy().view(np.uint16).astype(np.int64)
        x0 = x0 + rng.integers(-6, 7, x0.size)
        y0 = y0 + rng.integers(-6, 7, y0.size)
        far = rng.random(x0.size) < 0.05                     # predicted far outside the image
        x0[far] = 60000
        x0, y0 = np.clip(x0, 0, 65535), np.clip(y0, 0, 65535)
        kps["x0"].copy_(torch.from_numpy(x0.astype(np.uint16).view(np.int16)))
        kps["y0"].copy_(torch.from_numpy(y0.astype(np.uint16).view(np.int16)))
        n_max = fp.params.n_max
        refs = []
        for i in range(fp.n):
            r = dict(fp.results(i))
            n = len(r["x"])
            r["x0"] = x0[i * n_max:i * n_max + n].astype(np.uint16)
            r["y0"] = y0[i * n_max:i * n_max + n].astype(np.uint16)
            refs.append(r)
        # (the far points fall in the edge buckets; no query window reaches them)
        for st in SETTINGS + [(255, 11, 256, 0)]:
            say("case: feature_match map points", st)
            check(torch, fc, fp, kps, refs, st)
    finally:
        fp.close()
        fc.close()
