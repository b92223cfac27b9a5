"""Train and evaluate the learned cell proposer on the GPU.

Everything numeric runs in the library's kernels: the exact path labels
each generated pair (cells holding the native-scale position of a final
keypoint), cnn_forward / cnn_backward compute the weighted binary
cross-entropy gradient and cnn_adam_step updates the weights.  Scenes come
from the seeded generator (200 polygons, blur 1, noise 3, disparities
0..64) at 1241 x 376 ("kitti": training seeds 10^6 + i, held-out seeds
2 * 10^6 + i) or (800 polygons, disparities 0..128, at most 4000
keypoints) at 1920 x 1080 ("hd": 3 * 10^6 + i and 4 * 10^6 + i).  The
held-out pass picks the largest threshold whose gated path keeps >= 99%
of the exact path's keypoints, and does the same for a non-learned
baseline (level-3 intensity range per cell); thresholds are stored per
image size with the weights.

    python -m paper_2410_04090_amd.train --pairs 50000 --out proposer.npz
    python -m paper_2410_04090_amd.train --scene hd --init proposer.npz --pairs 8000 \\
        --batch 16 --out proposer_hd.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

class Scene:
    """Generator settings and detection parameters of one training domain."""

    def __init__(self, name, w, h, polys, max_disp, params_kw, seed_train, seed_eval):
        self.name, self.w, self.h, self.polys, self.max_disp = name, w, h, polys, max_disp
        self.params_kw, self.seed_train, self.seed_eval = params_kw, seed_train, seed_eval

    def params(self):
        from synth.configs import Params
        return Params(**self.params_kw)

    @property
    def size(self):
        return "%dx%d" % (self.w, self.h)


SCENES = {
    # KITTI-shaped pairs: 200 polygons, disparities 0..64, at most 2000 keypoints
    "kitti": Scene("kitti", 1241, 376, 200, 64, {}, 1_000_000, 2_000_000),
    # 1080p pairs: 800 polygons, disparities 0..128, at most 4000 keypoints
    "hd": Scene("hd", 1920, 1080, 800, 128, {"n_max": 4000, "d_max": 128}, 3_000_000, 4_000_000),
}


def _gen(job):
    from synth import scenes
    seed, w, h, polys, dmax = job
    return scenes.stereo_pair(seed, w, h, polys, dmax)


def pair_batches(scene, seed0, n_pairs, batch, procs):
    """Yield lists of `batch` pairs (left, right), generated in worker processes."""
    import multiprocessing as mp
    jobs = [(s, scene.w, scene.h, scene.polys, scene.max_disp) for s in range(seed0, seed0 + n_pairs)]
    with mp.get_context("fork").Pool(procs) as pool:
        buf = []
        for pair in pool.imap(_gen, jobs, chunksize=4):
            buf.append(pair)
            if len(buf) == batch:
                yield buf
                buf = []
    if buf:
        yield buf


class Proposer:
    """Frontend + proposer state for batches of same-size stereo pairs."""

    def __init__(self, scene, batch_pairs, init_seed=7, lr=2e-3):
        import torch
        from synth import pattern as pat
        from . import vsfe
        from .frontend import Frontend
        self.torch, self.vsfe = torch, vsfe
        self.scene = scene
        self.params = scene.params()
        self.fe = Frontend(self.params, [(scene.w, scene.h)] * (2 * batch_pairs), pat.brief_pattern())
        self.offs = self.fe.grid_offsets()
        theta = np.concatenate([p.reshape(-1) for p in pat.cnn_init(init_seed)]).astype(np.float32)
        dev = "cuda"
        self.w = torch.tensor(theta, device=dev)
        self.wb = self.w.to(torch.bfloat16).view(torch.int16).contiguous()
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.grad = torch.zeros_like(self.w)
        self.loss = torch.zeros(1, device=dev)
        self.targets = torch.zeros(int(self.fe.cnn.grid_elems), dtype=torch.float32, device=dev)
        self.step_no = 0
        self.lr = lr

    # ------------------------------------------------------------ labels
    def exact_keypoints(self):
        """Run the exact detection on the uploaded batch; per image (x0, y0, keys)."""
        fe = self.fe
        fe.run(describe=False)
        self.torch.cuda.synchronize()
        out = []
        counts = fe.kp_count.cpu().numpy()
        n_max = fe.params.n_max
        x0 = fe.kps["x0"].cpu().numpy().view(np.uint16)
        y0 = fe.kps["y0"].cpu().numpy().view(np.uint16)
        lv = fe.kps["level"].cpu().numpy()
        xx = fe.kps["x"].cpu().numpy().view(np.uint16)
        yy = fe.kps["y"].cpu().numpy().view(np.uint16)
        for i in range(fe.n):
            s = slice(i * n_max, i * n_max + int(counts[i]))
            keys = set(zip(lv[s].tolist(), xx[s].tolist(), yy[s].tolist()))
            out.append((x0[s], y0[s], keys))
        return out

    def set_targets(self, kps):
        from . import labels
        t = np.zeros(self.targets.numel(), np.float32)
        cells = []
        for i, (x0, y0, _) in enumerate(kps):
            W, H = self.scene.w, self.scene.h
            lab = labels.positive_cells(x0, y0, W, H)
            cells.append(lab)
            off, hz, wz = self.offs[i]
            t[off:off + hz * wz] = labels.grid_targets(lab, W, H, wz, hz).reshape(-1)
        self.targets.copy_(self.torch.from_numpy(t))
        return cells

    # ------------------------------------------------------------ training
    def train_step(self, pairs, total_steps, pos_weight=1.0):
        fe, vs = self.fe, self.vsfe
        imgs = [im for pr in pairs for im in pr]
        if len(imgs) < fe.n:        # last partial batch: repeat to fill
            imgs = (imgs * (fe.n // len(imgs) + 1))[:fe.n]
        fe.upload(imgs)
        self.set_targets(self.exact_keypoints())
        vs.cnn_forward(fe.ctx, fe.batch, fe.pyr, self.wb, fe.cnn_ws, fe.grid_logits, fe.status)
        vs.cnn_backward(fe.ctx, fe.batch, fe.pyr, self.wb, fe.cnn_ws, fe.grid_logits, self.targets, pos_weight,
                        self.grad, self.loss, fe.status)
        self.step_no += 1
        frac = self.step_no / max(total_steps, 1)
        lr = 1e-4 + 0.5 * (self.lr - 1e-4) * (1 + math.cos(math.pi * min(frac, 1.0)))
        vs.cnn_adam_step(self.w, self.wb, self.m, self.v, self.grad, lr, 0.9, 0.999, 1e-8, self.step_no)
        return float(self.loss.item())

    def save(self, path, meta):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        np.savez(path, params=self.w.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                 step=self.step_no, meta=json.dumps(meta))

    def load(self, path, weights_only=False):
        d = np.load(path, allow_pickle=False)
        self.w.copy_(self.torch.from_numpy(d["params"].astype(np.float32)))
        self.wb.copy_(self.w.to(self.torch.bfloat16).view(self.torch.int16))
        if "m" in d and not weights_only:
            self.m.copy_(self.torch.from_numpy(d["m"]))
            self.v.copy_(self.torch.from_numpy(d["v"]))
            self.step_no = int(d["step"])
        return json.loads(str(d["meta"])) if "meta" in d else {}

    # ------------------------------------------------------------ evaluation
    def gated_keypoints(self, mask_u8):
        fe = self.fe
        fe.cell_mask.copy_(self.torch.from_numpy(mask_u8))
        fe.run(mask=fe.cell_mask, describe=False)
        self.torch.cuda.synchronize()
        counts = fe.kp_count.cpu().numpy()
        n_max = fe.params.n_max
        lv = fe.kps["level"].cpu().numpy()
        xx = fe.kps["x"].cpu().numpy().view(np.uint16)
        yy = fe.kps["y"].cpu().numpy().view(np.uint16)
        return [set(zip(lv[i * n_max:i * n_max + int(counts[i])].tolist(),
                        xx[i * n_max:i * n_max + int(counts[i])].tolist(),
                        yy[i * n_max:i * n_max + int(counts[i])].tolist())) for i in range(fe.n)]


def evaluate(prop, n_pairs, batch, procs, n_tau=12):
    """Held-out recall / precision / kept-cell fraction for the CNN and the
    contrast baseline over candidate thresholds."""
    from . import labels
    fe, torch, vs, sc = prop.fe, prop.torch, prop.vsfe, prop.scene
    W, H = sc.w, sc.h
    batches = []
    for pairs in pair_batches(sc, sc.seed_eval, n_pairs, batch, procs):
        imgs = [im for pr in pairs for im in pr]
        if len(imgs) < fe.n:
            imgs = (imgs * (fe.n // len(imgs) + 1))[:fe.n]
        fe.upload(imgs)
        kps = prop.exact_keypoints()
        vs.cnn_propose(fe.ctx, fe.batch, fe.pyr, prop.wb, 0.0, fe.cnn_ws, fe.grid_logits, fe.cell_logits,
                       fe.cell_mask, fe.status)
        torch.cuda.synchronize()
        cl = fe.cell_logits.cpu().numpy().copy()
        con = np.concatenate([labels.contrast_scores(fe.pyramid_levels(i)[3], W, H).reshape(-1)
                              for i in range(fe.n)])
        pos = np.concatenate([labels.positive_cells(k[0], k[1], W, H).reshape(-1) for k in kps])
        batches.append((imgs, [k[2] for k in kps], cl, con, pos))
    all_cl = np.concatenate([b[2] for b in batches])
    all_con = np.concatenate([b[3] for b in batches])
    all_pos = np.concatenate([b[4] for b in batches]).astype(bool)

    def sweep(scores, cands):
        rows = []
        for tau in cands:
            got = ref_n = hit = kept = cells = 0
            for imgs, refs, cl, con, pos in batches:
                s = cl if scores == "cnn" else con
                mask = (s >= tau).astype(np.uint8)
                fe.upload(imgs)
                gk = prop.gated_keypoints(mask)
                for r, g in zip(refs, gk):
                    ref_n += len(r)
                    got += len(g)
                    hit += len(r & g)
                kept += int(mask.sum())
                cells += mask.size
            rows.append({"thresh": float(tau), "recall": hit / max(ref_n, 1), "precision": hit / max(got, 1),
                         "kept_frac": kept / max(cells, 1)})
        return rows

    qs = [0.0, 0.001, 0.002, 0.004, 0.007, 0.01, 0.015, 0.02, 0.03, 0.05, 0.08, 0.12][:n_tau]
    cnn_c = sorted(set(float(np.quantile(all_cl[all_pos], q)) for q in qs))
    con_c = sorted(set(float(np.quantile(all_con[all_pos], q)) for q in qs))
    res = {"cnn": sweep("cnn", cnn_c), "contrast": sweep("con", con_c), "pos_frac": float(all_pos.mean())}
    for k in ("cnn", "contrast"):
        ok = [r for r in res[k] if r["recall"] >= 0.99]
        res[k + "_chosen"] = max(ok, key=lambda r: r["thresh"]) if ok else None
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scene", default="kitti", choices=sorted(SCENES))
    ap.add_argument("--pairs", type=int, default=50000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--eval-pairs", type=int, default=1000)
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--pos-weight", type=float, default=1.0)
    ap.add_argument("--out", default="proposer.npz")
    ap.add_argument("--resume", default=None, help="continue from a checkpoint (weights + Adam state)")
    ap.add_argument("--init", default=None, help="start from a checkpoint's weights with a fresh optimizer")
    ap.add_argument("--eval-only", action="store_true")
    args = ap.parse_args()
    sc = SCENES[args.scene]
    prop = Proposer(sc, args.batch, lr=args.lr)
    meta = {}
    if args.resume:
        meta = prop.load(args.resume)
    elif args.init:
        meta = prop.load(args.init, weights_only=True)
    meta = dict(meta)
    t0 = time.time()
    if not args.eval_only:
        history = meta.pop("history", [])
        prev = {k: meta[k] for k in ("scene", "pairs", "train_seed0", "final_loss") if k in meta}
        if prev:
            history.append(prev)
        total = (args.pairs + args.batch - 1) // args.batch
        losses = []
        for k, pairs in enumerate(pair_batches(sc, sc.seed_train, args.pairs, args.batch, args.procs)):
            losses.append(prop.train_step(pairs, total, args.pos_weight))
            if (k + 1) % 50 == 0 or k + 1 == total:
                print("step %d/%d loss %.4f (%.0f s)" % (k + 1, total, float(np.mean(losses[-50:])), time.time() - t0),
                      flush=True)
            if (k + 1) % 500 == 0:
                prop.save(args.out, {"pairs_seen": (k + 1) * args.batch, "scene": sc.name})
        # new weights: earlier evaluations no longer apply
        meta = {"scene": sc.name, "pairs": args.pairs, "batch": args.batch, "lr": args.lr,
                "pos_weight": args.pos_weight, "train_seed0": sc.seed_train,
                "final_loss": float(np.mean(losses[-50:])) if losses else None, "train_seconds": time.time() - t0,
                "history": history}
    ev = evaluate(prop, args.eval_pairs, args.batch, args.procs)
    evals = dict(meta.get("evals", {}))
    evals[sc.size] = {"seed0": sc.seed_eval, "pairs": args.eval_pairs, **ev}
    meta["evals"] = evals
    meta["thresholds"] = {k: v["cnn_chosen"]["thresh"] for k, v in evals.items() if v.get("cnn_chosen")}
    prop.save(args.out, meta)
    print(json.dumps({"scene": sc.name, "eval": {k: ev[k] for k in ("pos_frac", "cnn_chosen", "contrast_chosen")}}),
          flush=True)


if __name__ == "__main__":
    main()
