"""The allocation-free aggregation entry point against the one with a
workspace: same keypoints and counts, bit for bit, on two calls in a row
(the second on a smaller batch, so the shared scratch still holds the first
call's ranks), and a clear capacity error past its fixed scratch."""
import numpy as np
import pytest

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


def _snapshot(torch, fe):
    torch.cuda.synchronize()
    out = {k: v.clone() for k, v in fe.kps.items()}
    out["count"] = fe.kp_count.clone()
    return out


def _run_both(torch, imgs, params):
    from paper_2410_04090_amd import vsfe
    from paper_2410_04090_amd.frontend import Frontend
    fe = Frontend(params, [(im.shape[1], im.shape[0]) for im in imgs], pat.brief_pattern())
    try:
        fe.upload(imgs)
        fe.run(describe=False)                  # pyramid, detection, aggregation with the workspace
        ref = _snapshot(torch, fe)
        for t in fe.kps.values():
            t.fill_(0x55)
        fe.kp_count.fill_(-7)
        vsfe.pyca_cull_aggregate_noalloc(fe.ctx, fe.batch, fe.cell_keys, fe.kps, fe.kp_count, fe.status)
        got = _snapshot(torch, fe)
        assert int(fe.status.item()) == 0
        counts = ref["count"].cpu().numpy()
        assert np.array_equal(counts, got["count"].cpu().numpy())
        n_max = params.n_max
        for k in fe.kps:
            a, b = ref[k].cpu().numpy(), got[k].cpu().numpy()
            for i, n in enumerate(counts):
                s = slice(i * n_max, i * n_max + int(n))
                assert np.array_equal(a[s], b[s]), (k, i)
        return int(counts.sum()), int(fe.info.n_cells)
    finally:
        fe.close()


def test_noalloc_matches_workspace_entry_point(torch_mod):
    torch = torch_mod
    big = []
    for s in (7001, 7002):
        big += list(scenes.stereo_pair(s, 1241, 376, 200, 64))
    say("case: noalloc aggregation, 4 x 1241x376")
    n1, c1 = _run_both(torch, big, Params())
    small = list(scenes.stereo_pair(7003, 640, 360, 120, 40))
    say("case: noalloc aggregation, 2 x 640x360 (second call, smaller batch)")
    n2, c2 = _run_both(torch, small, Params())
    assert n1 > 0 and n2 > 0 and c2 < c1


def test_noalloc_rejects_batches_past_its_scratch(torch_mod):
    from paper_2410_04090_amd import vsfe
    from paper_2410_04090_amd.frontend import Frontend
    torch = torch_mod
    # 5 images of 8192 x 8192 with 8-pixel cells on one level: 5 x 2^20 cells > 2^22
    n = 5
    p = Params(n_levels=1, cell0=8, n_max=16)
    say("case: noalloc capacity error, %d x 8192x8192, 8-pixel cells (no kernel runs)" % n)
    fe = Frontend(p, [(8192, 8192)] * n, pat.brief_pattern())
    try:
        assert fe.info.n_cells > vsfe.NOALLOC_MAX_CELLS
        with pytest.raises(vsfe.VsfeError) as e:
            vsfe.pyca_cull_aggregate_noalloc(fe.ctx, fe.batch, fe.cell_keys, fe.kps, fe.kp_count, fe.status)
        assert e.value.code == vsfe.ECAPACITY
        assert "at most" in str(e.value)
        torch.cuda.synchronize()
    finally:
        fe.close()
