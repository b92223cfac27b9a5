"""Bit-exact parity of stereo_refine (through the C ABI) with the oracle's
sub-pixel refinement, on the matches of the exact path: one KITTI-sized
pair, a mixed batch with ragged sizes (down to 97 x 61), window and radius
settings at both limits, and the smallest border the descriptors allow;
unmatched keypoints and minima at the end of the search range are the
not-refined cases that occur."""
import numpy as np
import pytest

import oracle
from synth import pattern as pat
from synth import scenes
from synth.configs import Params
from tests.parity_util import say

pytestmark = pytest.mark.gpu
INT32_MIN = -(2 ** 31)


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_case(torch, pairs, params, settings, layout=None):
    from paper_2410_04090_amd.frontend import Frontend
    imgs = [im for pr in pairs for im in pr]
    fe = Frontend(params, [(im.shape[1], im.shape[0]) for im in imgs], pat.brief_pattern(), layout=layout)
    try:
        fe.upload(imgs)
        fe.run()
        n_ref = 0
        for w, r in settings:
            say("case: refine sizes=%s w=%d r=%d" % ([im.shape for im in imgs[::2]], w, r))
            fe.refine(half_window=w, search_radius=r)
            torch.cuda.synchronize()
            assert int(fe.status.item()) == 0
            for p in range(len(pairs)):
                L, R = imgs[2 * p], imgs[2 * p + 1]
                H, W = L.shape
                kl, kr = fe.results(2 * p), fe.results(2 * p + 1)
                idx, _, _ = fe.matches(p)
                pl = oracle.pyramid_packed(L, params.n_levels)
                pr = oracle.pyramid_packed(R, params.n_levels)
                ref_d, ref_s = oracle.stereo_refine(pl, pr, W, H, kl, kr, idx, w, r)
                got_d, got_s = fe.refined(p)
                assert np.array_equal(ref_d, got_d), (p, w, r, int(np.argmax(ref_d != got_d)))
                assert np.array_equal(ref_s, got_s), (p, w, r)
                n_ref += int((ref_d != INT32_MIN).sum())
        return n_ref
    finally:
        fe.close()


def test_refine_pair_1241x376(torch_mod):
    pair = scenes.stereo_pair(8001, 1241, 376, 200, 64)
    n = run_case(torch_mod, [pair], Params(), [(5, 5)])
    assert n > 100


def test_refine_mixed_ragged_batch(torch_mod):
    pairs = [scenes.stereo_pair(8002, 640, 480, 150, 48), scenes.stereo_pair(8003, 333, 201, 60, 24),
             scenes.stereo_pair(8004, 97, 61, 10, 8)]
    run_case(torch_mod, pairs, Params(), [(5, 5), (1, 1), (7, 7), (3, 2)])


def test_refine_smallest_border_largest_window(torch_mod):
    # border 15 (the least the descriptors allow) with the largest window and
    # radius: windows reach the level edges (7 + 7 < 15)
    pair = scenes.stereo_pair(8005, 400, 256, 120, 40)
    n = run_case(torch_mod, [pair], Params(border=15), [(7, 7), (7, 1)])
    assert n > 0


@pytest.mark.parametrize("align", [1, 4])
def test_refine_unaligned_input_layout(torch_mod, align):
    """Level-0 rows not 4-byte aligned (align 1: byte reads) or 4-byte but
    not 16-byte aligned (align 4: dword reads)."""
    pairs = [scenes.stereo_pair(8006, 401, 257, 100, 30)]
    pitches, offsets, at = [], [], align
    for _ in range(2):
        pt = 401 + (3 if align == 1 else 7)
        pitches.append(pt)
        offsets.append(at)
        at += pt * 257 + (5 if align == 1 else 8)
    n = run_case(torch_mod, pairs, Params(), [(5, 5), (7, 7)], layout=(pitches, offsets))
    assert n > 0
