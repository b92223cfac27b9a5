"""What the trained cell proposer gains over the method without it.

On held-out 1080p pairs (seeds that neither training nor threshold
calibration used), the exact path (every cell kept) is compared with three
proposers gating the same exact detector:

* the packaged trained network at its packaged threshold;
* the same network with its initial (untrained) weights;
* a non-learned proposer: the level-3 intensity range over each cell.

Recall is measured by running the gated path and comparing its keypoints
(level, x, y) with the exact path's.  The untrained network and the
non-learned proposer get the largest threshold that reaches 99 % recall on
these very pairs, a choice that favours them.
"""
import os

import numpy as np
import pytest

from synth import pattern as pat
from synth import scenes
from synth.configs import Params
from tests.parity_util import say

pytestmark = pytest.mark.gpu

W, H = 1920, 1080
SEEDS = range(5_000_000, 5_000_004)
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2410_04090_amd", "weights",
                       "proposer_1920x1080.npz")


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def keypoint_sets(torch, fe):
    torch.cuda.synchronize()
    counts = fe.kp_count.cpu().numpy()
    n_max = fe.params.n_max
    lv = fe.kps["level"].cpu().numpy()
    xx = fe.kps["x"].cpu().numpy().view(np.uint16)
    yy = fe.kps["y"].cpu().numpy().view(np.uint16)
    x0 = fe.kps["x0"].cpu().numpy().view(np.uint16)
    y0 = fe.kps["y0"].cpu().numpy().view(np.uint16)
    keys, native = [], []
    for i in range(fe.n):
        s = slice(i * n_max, i * n_max + int(counts[i]))
        keys.append(set(zip(lv[s].tolist(), xx[s].tolist(), yy[s].tolist())))
        native.append((x0[s].copy(), y0[s].copy()))
    return keys, native


def gated_recall(torch, fe, exact, mask):
    fe.cell_mask.copy_(torch.from_numpy(mask.astype(np.uint8)))
    fe.run(mask=fe.cell_mask, describe=False)
    got, _ = keypoint_sets(torch, fe)
    ref_n = sum(len(r) for r in exact)
    hit = sum(len(r & g) for r, g in zip(exact, got))
    return hit / max(ref_n, 1), float(mask.mean())


def best_at_recall(torch, fe, exact, scores, pos, target=0.99):
    """Largest threshold (among low quantiles of the positive cells' scores)
    whose gated path reaches `target` recall: (threshold, recall, kept)."""
    cands = sorted({float(np.quantile(scores[pos], q)) for q in
                    (0.0, 0.001, 0.002, 0.004, 0.007, 0.01, 0.015, 0.02, 0.03, 0.05, 0.08, 0.12)}, reverse=True)
    for tau in cands:
        rec, kept = gated_recall(torch, fe, exact, scores >= tau)
        if rec >= target:
            return tau, rec, kept
    return None, 1.0, 1.0          # keep every cell: the method without a proposer


def test_trained_proposer_gain(torch_mod):
    torch = torch_mod
    from paper_2410_04090_amd import labels, vsfe
    from paper_2410_04090_amd.frontend import Frontend
    d = np.load(WEIGHTS, allow_pickle=False)
    import json
    meta = json.loads(str(d["meta"]))
    tau_trained = float(meta["thresholds"]["%dx%d" % (W, H)])
    theta_trained = d["params"].astype(np.float32)
    theta_init = np.concatenate([p.reshape(-1) for p in pat.cnn_init(7)]).astype(np.float32)

    imgs = [im for s in SEEDS for im in scenes.stereo_pair(s, W, H, 800, 128)]
    p = Params(n_max=4000, d_max=128)
    say("case: held-out 1080p pairs, seeds %d..%d" % (SEEDS[0], SEEDS[-1]))
    fe = Frontend(p, [(W, H)] * len(imgs), pat.brief_pattern())
    try:
        fe.upload(imgs)
        fe.run(describe=False)
        exact, native = keypoint_sets(torch, fe)
        pos = np.concatenate([labels.positive_cells(x0, y0, W, H).reshape(-1) for x0, y0 in native]).astype(bool)

        def logits(theta):
            wb = torch.from_numpy(theta).cuda().to(torch.bfloat16).view(torch.int16).contiguous()
            vsfe.cnn_propose(fe.ctx, fe.batch, fe.pyr, wb, 0.0, fe.cnn_ws, fe.grid_logits, fe.cell_logits,
                             fe.cell_mask, fe.status)
            torch.cuda.synchronize()
            return fe.cell_logits.cpu().numpy().copy()

        cl_trained = logits(theta_trained)
        rec_t, kept_t = gated_recall(torch, fe, exact, cl_trained >= tau_trained)
        _, rec_u, kept_u = best_at_recall(torch, fe, exact, logits(theta_init), pos)
        con = np.concatenate([labels.contrast_scores(fe.pyramid_levels(i)[3], W, H).reshape(-1)
                              for i in range(fe.n)])
        _, rec_c, kept_c = best_at_recall(torch, fe, exact, con, pos)
        say("cells holding a final keypoint: %.3f" % pos.mean())
        say("trained (packaged threshold): recall %.4f, cells kept %.3f" % (rec_t, kept_t))
        say("untrained, best threshold at 99%% recall: recall %.4f, cells kept %.3f" % (rec_u, kept_u))
        say("intensity range, best threshold at 99%% recall: recall %.4f, cells kept %.3f" % (rec_c, kept_c))
        # the calibrated threshold carries over to unseen pairs (measured 0.9929)
        assert rec_t >= 0.99
        # gain over the method without a proposer: a sizeable share of cells is skipped
        assert kept_t <= 0.85
        # and it comes from training: the untrained network, even with its
        # threshold picked on these pairs, keeps clearly more cells
        assert kept_t <= kept_u - 0.05
    finally:
        fe.close()


@pytest.mark.skip(reason="not met: on these held-out pairs the trained network keeps 70.2 % of the cells at "
                         "99.29 % recall, the non-learned level-3 intensity range 66.7 % at 99.16 % (its threshold "
                         "picked on the same pairs); the network does not beat that statistic on this workload")
def test_trained_proposer_beats_intensity_range(torch_mod):
    """The trained network should keep fewer cells than the intensity-range
    proposer at 99 % recall (kept_t < kept_c)."""
    torch = torch_mod
    from paper_2410_04090_amd import labels
    from paper_2410_04090_amd.frontend import Frontend
    d = np.load(WEIGHTS, allow_pickle=False)
    import json
    meta = json.loads(str(d["meta"]))
    tau_trained = float(meta["thresholds"]["%dx%d" % (W, H)])
    theta_trained = d["params"].astype(np.float32)
    imgs = [im for s in SEEDS for im in scenes.stereo_pair(s, W, H, 800, 128)]
    p = Params(n_max=4000, d_max=128)
    fe = Frontend(p, [(W, H)] * len(imgs), pat.brief_pattern())
    try:
        fe.upload(imgs)
        fe.run(describe=False)
        exact, native = keypoint_sets(torch, fe)
        pos = np.concatenate([labels.positive_cells(x0, y0, W, H).reshape(-1) for x0, y0 in native]).astype(bool)
        from paper_2410_04090_amd import vsfe
        wb = torch.from_numpy(theta_trained).cuda().to(torch.bfloat16).view(torch.int16).contiguous()
        vsfe.cnn_propose(fe.ctx, fe.batch, fe.pyr, wb, 0.0, fe.cnn_ws, fe.grid_logits, fe.cell_logits,
                         fe.cell_mask, fe.status)
        torch.cuda.synchronize()
        rec_t, kept_t = gated_recall(torch, fe, exact, fe.cell_logits.cpu().numpy() >= tau_trained)
        con = np.concatenate([labels.contrast_scores(fe.pyramid_levels(i)[3], W, H).reshape(-1)
                              for i in range(fe.n)])
        _, rec_c, kept_c = best_at_recall(torch, fe, exact, con, pos)
        assert rec_t >= 0.99 and kept_t < kept_c
    finally:
        fe.close()
