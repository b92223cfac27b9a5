"""GPU parity of the learned cell proposer with its oracle.

The network evaluated is the one with bfloat16-valued weights.  Its GPU
logits must match the oracle's float64 forward of the same weights with
unrounded activations (a float32-or-better CPU forward) within 1e-2
absolute, for random and for the packaged trained networks, both from the
inference kernel (float16 activations) and from the training forward
(bfloat16 value + remainder pairs, within 1e-3); cell logits and masks are
exact functions of the grid logits;
every gradient entry and the loss match the float64 oracle backward to a
stated tolerance; the gated exact path matches the oracle run on the
GPU's mask bit for bit, also for the benchmark's 1080p learned leg.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import cnn as ocnn
from synth import pattern as pat
from synth import scenes
from synth.configs import Params
from tests.parity_util import compare_kps, compare_matches, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2410_04090_amd", "weights")
LOGIT_TOL = 1e-2            # absolute, against the float64 forward of the same weights
TRAIN_LOGIT_TOL = 1e-3      # the training forward (value + remainder pairs), same reference
GRAD_RTOL = 1e-3            # per gradient entry, relative to the entry
GRAD_ATOL = 1e-4            # per gradient entry, relative to the layer's largest entry

LAYERS = [("w1", 0, 144), ("b1", 144, 160), ("w2", 160, 4768), ("b2", 4768, 4800), ("w3", 4800, 14016),
          ("b3", 14016, 14048), ("w4", 14048, 14080), ("b4", 14080, 14081)]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def theta_for(seed):
    """bfloat16-valued test weights (the kernels read the bfloat16 copy)."""
    rng = np.random.default_rng(seed)
    th = np.concatenate([p.reshape(-1) for p in pat.cnn_init(seed)]).astype(np.float64)
    # non-zero biases so that every ReLU regime is exercised
    for name, a, b in LAYERS:
        if name.startswith("b"):
            th[a:b] = rng.normal(0, 0.1, b - a)
    return ocnn.bf16_round(th)


def packaged(size):
    d = np.load(os.path.join(WEIGHTS, "proposer_%s.npz" % size), allow_pickle=False)
    return d["params"].astype(np.float64), json.loads(str(d["meta"]))


def bf16_tensor(torch, theta):
    return torch.tensor(theta, dtype=torch.float32).to(torch.bfloat16).view(torch.int16).cuda()


def make_batch(torch, imgs, params):
    from paper_2410_04090_amd.frontend import Frontend
    fe = Frontend(params, [(im.shape[1], im.shape[0]) for im in imgs], pat.brief_pattern())
    fe.upload(imgs)
    return fe


def grid_of(fe, z_all, i):
    off, hz, wz = fe.grid_offsets()[i]
    return z_all[off:off + hz * wz].reshape(hz, wz)


def images_mixed():
    a, b = scenes.stereo_pair(4001, 1241, 376, 200, 64)
    c = scenes.random_image(4002, 333, 201)
    return [a, b, c, scenes.mono_image(4003, 333, 201, 60)]


def test_forward_matches_oracle(torch_mod):
    torch = torch_mod
    imgs = images_mixed()
    p = Params()
    theta = theta_for(11)
    fe = make_batch(torch, imgs, p)
    try:
        say("cnn forward on", [im.shape for im in imgs])
        fe.run(describe=False)
        w = bf16_tensor(torch, theta)
        from paper_2410_04090_amd import vsfe
        vsfe.cnn_forward(fe.ctx, fe.batch, fe.pyr, w, fe.cnn_ws, fe.grid_logits, fe.status)
        torch.cuda.synchronize()
        z = fe.grid_logits.cpu().numpy()
        for i, img in enumerate(imgs):
            lv3 = oracle.pyramid(img, 4)[3]
            ref, _ = ocnn.forward(lv3, theta, bf16=False)
            got = grid_of(fe, z, i)
            assert got.shape == ref.shape
            err = np.abs(got - ref).max()
            say("image", i, "max |dz| vs float64 forward =", err, "range", ref.min(), ref.max())
            assert err <= LOGIT_TOL
            assert np.std(ref) > 0.05          # the test network is not degenerate
    finally:
        fe.close()


@pytest.mark.parametrize("size,W,H,polys,dmax", [("1241x376", 1241, 376, 200, 64),
                                                 ("1920x1080", 1920, 1080, 800, 128)])
def test_trained_network_logits_match_float64_forward(torch_mod, size, W, H, polys, dmax):
    """The packaged trained networks (larger logits than a random one) stay
    within the tolerance of the float64 forward on scenes of their size."""
    torch = torch_mod
    theta, _ = packaged(size)
    assert np.array_equal(theta, ocnn.bf16_round(theta))      # packaged weights are bfloat16 values
    imgs = list(scenes.stereo_pair(6001, W, H, polys, dmax))
    fe = make_batch(torch, imgs, Params())
    try:
        from paper_2410_04090_amd import vsfe
        fe.run(describe=False)
        w = bf16_tensor(torch, theta)
        vsfe.cnn_propose(fe.ctx, fe.batch, fe.pyr, w, 0.0, fe.cnn_ws, fe.grid_logits, fe.cell_logits, fe.cell_mask,
                         fe.status)
        torch.cuda.synchronize()
        z = fe.grid_logits.cpu().numpy()
        for i, img in enumerate(imgs):
            ref, _ = ocnn.forward(oracle.pyramid(img, 4)[3], theta, bf16=False)
            err = np.abs(grid_of(fe, z, i) - ref).max()
            say(size, "image", i, "max |dz| =", err, "range", ref.min(), ref.max())
            assert err <= LOGIT_TOL
    finally:
        fe.close()


def test_inference_is_deterministic(torch_mod):
    """Three cnn_propose calls on a 1080p pair give the same logits bit for
    bit (matrix-core products read too early differ from run to run in
    their later output columns), and they match the float64 forward."""
    torch = torch_mod
    theta, _ = packaged("1920x1080")
    imgs = list(scenes.stereo_pair(6002, 1920, 1080, 800, 128))
    fe = make_batch(torch, imgs, Params())
    try:
        from paper_2410_04090_amd import vsfe
        fe.run(describe=False)
        w = bf16_tensor(torch, theta)
        zs = []
        for _ in range(3):
            fe.grid_logits.fill_(float("nan"))
            vsfe.cnn_propose(fe.ctx, fe.batch, fe.pyr, w, 0.0, fe.cnn_ws, fe.grid_logits, fe.cell_logits,
                             fe.cell_mask, fe.status)
            torch.cuda.synchronize()
            zs.append(fe.grid_logits.cpu().numpy().copy())
        for z in zs[1:]:
            assert np.array_equal(zs[0].view(np.uint32), z.view(np.uint32))
        ref, _ = ocnn.forward(oracle.pyramid(imgs[1], 4)[3], theta, bf16=False)
        err = np.abs(grid_of(fe, zs[0], 1) - ref).max()
        say("repeated 1080p inference: identical; max |dz| =", err)
        assert err <= LOGIT_TOL
    finally:
        fe.close()


def test_propose_cells_and_mask(torch_mod):
    torch = torch_mod
    imgs = images_mixed()[:2]
    p = Params()
    theta = theta_for(12)
    fe = make_batch(torch, imgs, p)
    try:
        from paper_2410_04090_amd import vsfe
        fe.run(describe=False)
        w = bf16_tensor(torch, theta)
        z_all = None
        for thresh in (-0.5, 0.0, 0.7):
            vsfe.cnn_propose(fe.ctx, fe.batch, fe.pyr, w, thresh, fe.cnn_ws, fe.grid_logits, fe.cell_logits,
                             fe.cell_mask, fe.status)
            torch.cuda.synchronize()
            z_all = fe.grid_logits.cpu().numpy()
            cl = fe.cell_logits.cpu().numpy()
            mk = fe.cell_mask.cpu().numpy()
            at = 0
            for i, img in enumerate(imgs):
                H, W = img.shape
                ref = ocnn.cell_logits(grid_of(fe, z_all, i), W, H).reshape(-1)
                got = cl[at:at + ref.size]
                assert np.array_equal(got, ref.astype(np.float32))
                assert np.array_equal(mk[at:at + ref.size], (ref >= thresh).astype(np.uint8))
                at += ref.size
    finally:
        fe.close()


def test_fused_inference_and_training_forward_match_oracle(torch_mod):
    """cnn_propose (the persistent fused kernel, float16 activations in LDS)
    and cnn_forward (layer by layer through HBM, bfloat16 value + remainder
    pairs) both match the float64 forward: the inference logits within 1e-2,
    the training logits within 1e-3; sizes include tiles cut by every
    border and an image smaller than one tile."""
    torch = torch_mod
    imgs = images_mixed() + [scenes.random_image(4004, 61, 47), scenes.mono_image(4005, 203, 333, 40)]
    p = Params()
    theta = theta_for(15)
    fe = make_batch(torch, imgs, p)
    try:
        from paper_2410_04090_amd import vsfe
        fe.run(describe=False)
        w = bf16_tensor(torch, theta)
        vsfe.cnn_forward(fe.ctx, fe.batch, fe.pyr, w, fe.cnn_ws, fe.grid_logits, fe.status)
        torch.cuda.synchronize()
        z_fwd = fe.grid_logits.cpu().numpy().copy()
        fe.grid_logits.fill_(float("nan"))
        vsfe.cnn_propose(fe.ctx, fe.batch, fe.pyr, w, 0.0, fe.cnn_ws, fe.grid_logits, fe.cell_logits, fe.cell_mask,
                         fe.status)
        torch.cuda.synchronize()
        z_fused = fe.grid_logits.cpu().numpy()
        assert np.isfinite(z_fused).all()
        for i, img in enumerate(imgs):
            ref, _ = ocnn.forward(oracle.pyramid(img, 4)[3], theta, bf16=False)
            e_inf = np.abs(grid_of(fe, z_fused, i) - ref).max()
            e_tr = np.abs(grid_of(fe, z_fwd, i) - ref).max()
            say("image", i, img.shape, "max |dz| vs float64 forward: inference", e_inf, "training", e_tr)
            assert e_inf <= LOGIT_TOL
            assert e_tr <= TRAIN_LOGIT_TOL
    finally:
        fe.close()


def test_backward_matches_oracle(torch_mod):
    torch = torch_mod
    imgs = [scenes.mono_image(4010, 640, 480, 120), scenes.random_image(4011, 420, 300)]
    p = Params()
    theta = theta_for(13)
    fe = make_batch(torch, imgs, p)
    try:
        from paper_2410_04090_amd import vsfe
        fe.run(describe=False)
        w = bf16_tensor(torch, theta)
        vsfe.cnn_forward(fe.ctx, fe.batch, fe.pyr, w, fe.cnn_ws, fe.grid_logits, fe.status)
        rng = np.random.default_rng(3)
        n = int(fe.cnn.grid_elems)
        t = (rng.random(n) < 0.6).astype(np.float32)
        tgt = torch.tensor(t).cuda()
        grad = torch.zeros(ocnn.N_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        vsfe.cnn_backward(fe.ctx, fe.batch, fe.pyr, w, fe.cnn_ws, fe.grid_logits, tgt, 1.7, grad, loss, fe.status)
        torch.cuda.synchronize()
        g_gpu = grad.cpu().numpy().astype(np.float64)
        # oracle: mean BCE over all positions of the batch
        zs, caches = [], []
        for img in imgs:
            z, cache = ocnn.forward(oracle.pyramid(img, 4)[3], theta, bf16=False)
            zs.append(z)
            caches.append(cache)
        zcat = np.concatenate([z.reshape(-1) for z in zs])
        ref_loss, dz = ocnn.bce_with_logits(zcat, t, pos_weight=1.7)
        g_ref = np.zeros(ocnn.N_PARAMS)
        at = 0
        for z, cache in zip(zs, caches):
            g_ref += ocnn.backward(cache, dz[at:at + z.size].reshape(z.shape))
            at += z.size
        say("loss gpu", float(loss.item()), "oracle", ref_loss)
        assert abs(float(loss.item()) - ref_loss) <= 1e-4 * ref_loss
        # every entry: |g_gpu - g_ref| <= ATOL * max|g_ref of the layer| + RTOL * |g_ref|
        # (float32 sums over ~10^5 positions against float64)
        for name, a, b in LAYERS:
            ref, got = g_ref[a:b], g_gpu[a:b]
            scale = np.abs(ref).max()
            bound = GRAD_ATOL * scale + GRAD_RTOL * np.abs(ref)
            bad = np.abs(got - ref) > bound
            worst = float(np.max(np.abs(got - ref) / (scale + 1e-30)))
            say("grad", name, "worst |dg| / max|g| =", worst, "entries out of bound:", int(bad.sum()))
            assert not bad.any(), (name, int(np.argmax(bad)), got[bad][:3], ref[bad][:3])
        # deterministic: a second backward gives the same bits
        grad2 = torch.zeros_like(grad)
        vsfe.cnn_backward(fe.ctx, fe.batch, fe.pyr, w, fe.cnn_ws, fe.grid_logits, tgt, 1.7, grad2, loss, fe.status)
        torch.cuda.synchronize()
        assert torch.equal(grad, grad2)
    finally:
        fe.close()


def test_adam_step(torch_mod):
    torch = torch_mod
    from paper_2410_04090_amd import vsfe
    rng = np.random.default_rng(4)
    n = ocnn.N_PARAMS
    w0 = rng.normal(size=n).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    w = torch.tensor(w0).cuda()
    wb = torch.zeros(n, dtype=torch.int16, device="cuda")
    m = torch.zeros(n, device="cuda")
    v = torch.zeros(n, device="cuda")
    gt = torch.tensor(g).cuda()
    mm, vv, ww = np.zeros(n), np.zeros(n), w0.astype(np.float64)
    for step in (1, 2, 3):
        vsfe.cnn_adam_step(w, wb, m, v, gt, 1e-3, 0.9, 0.999, 1e-8, step)
        mm = 0.9 * mm + 0.1 * g
        vv = 0.999 * vv + 0.001 * g.astype(np.float64) ** 2
        ww = ww - 1e-3 * (mm / (1 - 0.9 ** step)) / (np.sqrt(vv / (1 - 0.999 ** step)) + 1e-8)
    torch.cuda.synchronize()
    assert np.allclose(w.cpu().numpy(), ww, atol=1e-5)
    assert np.array_equal(wb.view(torch.bfloat16).float().cpu().numpy(),
                          ocnn.bf16_round(w.cpu().numpy()).astype(np.float32))


def test_learned_path_matches_oracle_on_gpu_mask(torch_mod):
    """The gated exact path equals the oracle run with the GPU's cell mask."""
    torch = torch_mod
    l, r = scenes.stereo_pair(4020, 640, 360, 120, 40)
    p = Params()
    theta = theta_for(14)
    fe = make_batch(torch, [l, r], p)
    try:
        w = bf16_tensor(torch, theta)
        fe.run_learned(w, 0.0)
        torch.cuda.synchronize()
        cl = fe.cell_logits.cpu().numpy()
        tau = float(np.median(cl[np.isfinite(cl)]))      # keeps about half of the cells
        fe.run_learned(w, tau)
        torch.cuda.synchronize()
        mk = fe.cell_mask.cpu().numpy()
        at = 0
        refs = []
        for i, img in enumerate((l, r)):
            ncx, ncy = (640 + 31) // 32, (360 + 31) // 32
            m0 = mk[at:at + ncx * ncy].reshape(ncy, ncx)
            at += ncx * ncy
            assert 0 < m0.sum() < m0.size          # a real gate: some cells on, some off
            _, ref = oracle.frontend_image(img, p, pat.brief_pattern(), cell_mask0=m0)
            compare_kps(ref, fe.results(i), i)
            refs.append(ref)
        compare_matches(fe, 0, refs[0], refs[1], p)
    finally:
        fe.close()


def test_learned_leg_1080p_matches_oracle_on_gpu_mask(torch_mod):
    """The benchmark's learned leg at its size: two 1920 x 1080 pairs of the
    1080p batch (seeds 200, 201), the packaged 1080p network at its
    packaged threshold, 4000 keypoints, disparities up to 128; the gated
    path (keypoints, descriptors, matches) equals the oracle fed the GPU's
    cell mask."""
    torch = torch_mod
    theta, meta = packaged("1920x1080")
    tau = float(meta["thresholds"]["1920x1080"])
    imgs = []
    for seed in (200, 201):
        imgs += list(scenes.stereo_pair(seed, 1920, 1080, 800, 128))
    p = Params(n_max=4000, d_max=128)
    fe = make_batch(torch, imgs, p)
    try:
        w = bf16_tensor(torch, theta)
        say("case: learned leg 1080p, seeds 200-201, tau", tau)
        fe.run_learned(w, tau)
        torch.cuda.synchronize()
        assert int(fe.status.item()) == 0
        mk = fe.cell_mask.cpu().numpy()
        ncx, ncy = 1920 // 32, (1080 + 31) // 32
        kept = mk[:4 * ncx * ncy].mean()
        say("kept cell fraction", kept)
        assert 0.3 < kept < 0.95                  # a real gate
        refs = []
        for i, img in enumerate(imgs):
            m0 = mk[i * ncx * ncy:(i + 1) * ncx * ncy].reshape(ncy, ncx)
            _, ref = oracle.frontend_image(img, p, pat.brief_pattern(), cell_mask0=m0)
            compare_kps(ref, fe.results(i), i)
            refs.append(ref)
        for pr in range(2):
            compare_matches(fe, pr, refs[2 * pr], refs[2 * pr + 1], p)
    finally:
        fe.close()
