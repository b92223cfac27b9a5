"""Bit-exact parity of fc_cull_crf (Feature Culling over the materialised
response matrix with the paper's thread schemes: MLPT + TEWA, log2
reduction, MLPT with one block per cell) with the oracle's culling at the
paper's cell sizes (23, 17, 13, 7, 3 and 32) on several pyramid levels and
ragged image sizes; and the culled keys equal the fused detector's at the
batch's own cells (no fallback threshold)."""
from dataclasses import replace

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


@pytest.fixture(scope="module")
def batch(torch_mod):
    from paper_2410_04090_amd.frontend import Frontend
    imgs = [scenes.mono_image(9101, 1241, 376, 200), scenes.random_image(9102, 640, 480),
            scenes.mono_image(9103, 333, 201, 60)]
    p = Params(eps_lo=-1)
    fe = Frontend(p, [(im.shape[1], im.shape[0]) for im in imgs], pat.brief_pattern(), with_crf=True)
    fe.upload(imgs)
    fe.run(describe=False)
    torch_mod.cuda.synchronize()
    yield fe, imgs, p
    fe.close()


def cull(torch, fe, level, cell, scheme, n_loc):
    from paper_2410_04090_amd import vsfe
    stride = vsfe.fc_cull_stride(fe.batch, level, cell)
    keys = torch.full((max(stride * fe.n, 1),), -1, dtype=torch.int32, device="cuda")
    vsfe.fc_cull_crf(fe.ctx, fe.batch, fe.crf, level, cell, scheme, n_loc, keys, fe.status)
    torch.cuda.synchronize()
    return keys.cpu().numpy().view(np.uint32), stride


@pytest.mark.parametrize("cell", [23, 17, 13, 7, 3, 32])
def test_schemes_match_oracle_culling(torch_mod, batch, cell):
    fe, imgs, p = batch
    for level in (0, 2, 5):
        levels = [oracle.pyramid(im, p.n_levels)[level] for im in imgs]
        refs = [oracle.cull_level(lv, cell, p)[0] for lv in levels]
        for scheme, n_loc in ((0, max(1, -(-cell // 8))), (0, 5), (1, 1), (2, 4), (2, max(1, -(-cell // 8)))):
            if scheme != 1 and -(-cell // n_loc) > 8:
                continue
            say("case: fc scheme", scheme, "cell", cell, "level", level, "n_loc", n_loc)
            keys, stride = cull(torch_mod, fe, level, cell, scheme, n_loc)
            for i, ref in enumerate(refs):
                got = keys[i * stride:i * stride + ref.size].reshape(ref.shape)
                assert np.array_equal(ref, got), (i, scheme, cell, level, int(np.argmax(ref.reshape(-1) != got.reshape(-1))))
            assert any(r.any() for r in refs)


def test_mlpt_equals_fused_detector_keys(torch_mod, batch):
    fe, imgs, p = batch
    for level in range(p.n_levels):
        c = oracle.cell_size(p.cell0, level)
        keys, stride = cull(torch_mod, fe, level, c, 0, max(1, -(-c // 8)))
        for i in range(fe.n):
            fused = fe.cell_keys_level(i, level)
            got = keys[i * stride:i * stride + fused.size].reshape(fused.shape)
            assert np.array_equal(fused, got), (i, level)


def test_undersized_keys_are_refused(torch_mod, batch):
    """The keys buffer a (level, cell) needs depends on both; one entry
    short is refused before any launch and the buffer is left untouched."""
    from paper_2410_04090_amd import vsfe
    fe, imgs, p = batch
    for level, cell in ((0, 3), (2, 7), (5, 32)):
        need = vsfe.fc_cull_stride(fe.batch, level, cell) * fe.n
        keys = torch_mod.full((need - 1,), -1, dtype=torch_mod.int32, device="cuda")
        with pytest.raises(vsfe.VsfeError) as ei:
            vsfe.fc_cull_crf(fe.ctx, fe.batch, fe.crf, level, cell, 0, 1 if cell <= 8 else -(-cell // 8), keys,
                             fe.status)
        assert ei.value.code == vsfe.ECAPACITY
        torch_mod.cuda.synchronize()
        assert (keys == -1).all()
