"""The repeatability harness on the GPU: the library's response dumps give
exactly the oracle's responses (so the F1 scores are the oracle's), and
Bounded Rectification scores at least plain FAST-9 on every angle's mean
over the scenes, with a rotation-stable F1."""
import numpy as np
import pytest

import oracle
from paper_2410_04090_amd import repeatability as R
from tests.parity_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_harness_matches_oracle_and_br_helps(torch_mod):
    seeds = (1, 2)
    cases = R.scene_images(seeds, R.ANGLES, 480)
    imgs = [c[2] for c in cases]
    say("case: repeatability, scenes %s, %d angles" % (seeds, len(R.ANGLES)))
    rb = R.responses_gpu(imgs, 20, 13)
    rp = R.responses_gpu(imgs, 20, 16)
    for img, a, b in zip(imgs, rb, rp):
        assert np.array_equal(a, oracle.crf(img, 20, 9, 13, 3))
        assert np.array_equal(b, oracle.crf(img, 20, 9, 16, 3))
    per = R.evaluate(cases, rb, rp, 3.0)
    f_br = np.array([per[a]["br"]["f1"] for a in per])
    f_pl = np.array([per[a]["plain"]["f1"] for a in per])
    say("F1 bounded rectification: mean %.3f min %.3f max %.3f" % (f_br.mean(), f_br.min(), f_br.max()))
    say("F1 plain FAST-9:          mean %.3f min %.3f max %.3f" % (f_pl.mean(), f_pl.min(), f_pl.max()))
    assert f_br.mean() > f_pl.mean()
    assert f_br.max() - f_br.min() < 0.1          # stable under rotation
