#!/usr/bin/env python3
"""Throughput benchmark of the stereo front-end on one MI355X.

One step = one pass of the whole exact path (pyramid, FAST + Bounded
Rectification with fused culling, pyramidal aggregation + cap, ORB
orientation + rBRIEF, stereo matching) over one batch of synthetic stereo
pairs already resident in HBM, replayed as one HIP graph.  Prints one JSON
line with the throughput, the dominant kernel's roofline figures (its
algorithmic bytes per launch over its measured launch time, and the HBM
bytes from the stored counter summary) and the oracle's host-core rate.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "stereo frames/s, exact vs learned-proposal path at ≥99% keypoint recall"
HBM_PEAK_GBS = 8000.0
PKG = os.path.join(ROOT, "paper_2410_04090_amd")
# source file of each call's kernels (a stored counter reading is valid only
# for the source it was taken from)
CALL_SOURCE = {"pyramid_build": "pyramid.hip", "fast_br_detect": "detect.hip", "pyca_cull_aggregate": "pyca.hip",
               "orb_describe": "orb.hip", "stereo_match": "stereo.hip"}


def _gen_pair(args):
    from synth import scenes
    seed, w, h, npoly, dmax = args
    return scenes.stereo_pair(seed, w, h, npoly, dmax)


def make_images(wl, procs):
    jobs = [(s, w, h, wl.n_polygons, wl.max_disparity) for (w, h), s in zip(wl.sizes, wl.seeds)]
    if procs > 1 and len(jobs) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(procs, len(jobs))) as pool:
            pairs = pool.map(_gen_pair, jobs)
    else:
        pairs = [_gen_pair(j) for j in jobs]
    imgs = []
    for l, r in pairs:
        imgs += [l, r]
    return imgs


def level_sizes(w, h, L):
    out = []
    for l in range(L):
        out.append(((2 * w * 5 ** l + 6 ** l) // (2 * 6 ** l), (2 * h * 5 ** l + 6 ** l) // (2 * 6 ** l)))
    return out


def time_call(fn, reps, stream):
    """Average duration (us) of fn() launched reps times back to back on
    `stream`, from HIP events recorded on that stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1000.0 / reps


def source_sha(call):
    import hashlib
    paths = [os.path.join(PKG, "csrc", CALL_SOURCE[call]), os.path.join(PKG, "csrc", "vsfe_internal.h")]
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(call, workload):
    """HBM bytes per launch of `call` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a copy-kernel calibration), or None
    when there is none or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.txt" % (call, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_sha(call):
        return None
    try:
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stored_counters(call, workload):
    """SQ instruction counts per launch of `call` from the committed counter
    summary (profiles/<call>_<workload>_sq.txt), or None when there is none
    or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_sq.txt" % (call, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_sha(call):
        return None
    try:
        return {k: float(kv[k]) for k in ("insts_valu_per_launch", "insts_salu_per_launch", "insts_lds_per_launch")}
    except (KeyError, ValueError):
        return None


def stored_ceiling():
    """VALU issue rate measured by the probe kernel (wave instructions/s)
    from profiles/ceiling_probe_mi355x.txt, or None when absent or the probe
    source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "ceiling_probe_mi355x.txt")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ("probe.hip", "vsfe_internal.h"):
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(fh.read())
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.split("(")[0].strip()
    if kv.get("source_sha") != h.hexdigest()[:16]:
        return None
    try:
        return float(kv["valu_wave_insts_per_s"])
    except (KeyError, ValueError):
        return None


# VALU issue peak: one wave64 instruction per SIMD every 4 cycles (16 lanes
# per SIMD), 4 SIMDs per CU, 256 CUs at 2.4 GHz: 256 x 4 x 2.4e9 / 4 =
# 614 G wave-instructions/s = 39.3 T lane-operations/s
VALU_WAVE_INSTS_PER_S = 256 * 4 * 2.4e9 / 4
VALU_LANE_OPS_PEAK_T = VALU_WAVE_INSTS_PER_S * 64 / 1e12


def copy_probe(mib):
    """A plain device-to-device copy of known size, for scaling the HBM
    byte counters (run under the counter profiler)."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "launches": 5}), flush=True)


def ceiling_probe():
    """Measured VALU issue rate and LDS read bandwidth of the device (the
    library's probe kernels), against the figures the roofline assumes."""
    import torch
    from paper_2410_04090_amd import vsfe
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"cus": n_cu}
    for kind, name, iters in ((vsfe.PROBE_VALU, "valu", 2000), (vsfe.PROBE_LDS, "lds", 4000)):
        blocks = n_cu * 8
        sink = torch.zeros(blocks * 256, dtype=torch.int32, device="cuda")
        clocks = torch.zeros(2, dtype=torch.int64, device="cuda")
        st = torch.cuda.current_stream()
        vsfe.probe(kind, blocks, iters // 10, sink, clocks, st)   # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record(st)
        for _ in range(reps):
            vsfe.probe(kind, blocks, iters, sink, clocks, st)
        e1.record(st)
        e1.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        cyc, wall = clocks.cpu().tolist()
        ghz = cyc / (wall / 100e6) / 1e9 if wall else None
        waves = blocks * 4
        if kind == vsfe.PROBE_VALU:
            insts = waves * 128 * iters
            rate = insts / sec
            out[name] = {"wave_insts": insts, "us": round(sec * 1e6, 1), "wave_insts_per_s": round(rate / 1e9, 1),
                         "unit": "G/s", "assumed_peak": round(VALU_WAVE_INSTS_PER_S / 1e9, 1),
                         "frac_of_assumed": round(rate / VALU_WAVE_INSTS_PER_S, 3), "sclk_ghz": round(ghz, 3) if ghz else None}
        else:
            nbytes = waves * 64 * 16 * 16 * iters
            bw = nbytes / sec
            out[name] = {"bytes": nbytes, "us": round(sec * 1e6, 1), "bytes_per_s": round(bw / 1e12, 2), "unit": "TB/s",
                         "bytes_per_clk_per_cu": round(bw / (n_cu * (ghz or 2.4) * 1e9), 1),
                         "sclk_ghz": round(ghz, 3) if ghz else None}
    print(json.dumps({"ceiling_probe": out}), flush=True)


def load_proposer(path):
    d = np.load(path, allow_pickle=False)
    meta = json.loads(str(d["meta"])) if "meta" in d else {}
    return d["params"].astype(np.float32), meta


def keypoint_sets(fe):
    import torch
    torch.cuda.synchronize()
    counts = fe.kp_count.cpu().numpy()
    n_max = fe.params.n_max
    lv = fe.kps["level"].cpu().numpy()
    xx = fe.kps["x"].cpu().numpy().view(np.uint16)
    yy = fe.kps["y"].cpu().numpy().view(np.uint16)
    out = []
    for i in range(fe.n):
        s = slice(i * n_max, i * n_max + int(counts[i]))
        out.append(set(zip(lv[s].tolist(), xx[s].tolist(), yy[s].tolist())))
    return out


_CPU_JOB = None


def _cpu_pair(i):
    import oracle
    wl, imgs, pattern = _CPU_JOB
    oracle.frontend_pair_native(imgs[2 * i], imgs[2 * i + 1], wl.params, pattern)
    return i


def cpu_baseline(wl, imgs, pattern, budget_s, procs=1):
    """The oracle on the first pairs of the batch, one pair per process at a
    time over `procs` processes, until the time budget is spent."""
    import oracle
    global _CPU_JOB
    n_pairs = len(imgs) // 2
    t0 = time.perf_counter()
    done = 0
    if procs <= 1:
        while done < n_pairs:
            oracle.frontend_pair_native(imgs[2 * done], imgs[2 * done + 1], wl.params, pattern)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
    else:
        import multiprocessing as mp
        _CPU_JOB = (wl, imgs, pattern)
        with mp.get_context("fork").Pool(procs) as pool:
            while done < n_pairs and time.perf_counter() - t0 <= budget_s:
                batch = list(range(done, min(n_pairs, done + procs)))
                pool.map(_cpu_pair, batch)
                done += len(batch)
        _CPU_JOB = None
    dt = time.perf_counter() - t0
    sizes = sorted(set(wl.sizes[:max(done, 1)]))
    what = "x".join(map(str, sizes[0])) if len(sizes) == 1 else "mixed sizes"
    how = "one thread" if procs <= 1 else "%d processes, one pair each at a time" % procs
    return {"value": done / dt, "unit": "stereo pairs/s", "cores": max(1, procs), "kind": "oracle",
            "sample": "%d of the %d pairs (%s), plain C oracle, %s, %.1f s" % (done, n_pairs, what, how, dt)}


def learned_path(args, fe, sizes, stream, exact_value):
    """Learned-proposal path on the same batch: CNN cell proposal on level 3,
    detection only in proposed cells, the rest unchanged.  Recall and
    precision are measured against the exact path's keypoints of this batch;
    the threshold was calibrated on held-out scenes of the same size."""
    import torch
    from paper_2410_04090_amd import vsfe
    if len(set(sizes)) != 1 or fe.cell_mask is None:
        return None
    w, h = sizes[0]
    path = args.proposer or os.path.join(PKG, "weights", "proposer_%dx%d.npz" % (w, h))
    if not os.path.exists(path):
        print("no proposer weights for %dx%d, learned path skipped" % (w, h), file=sys.stderr, flush=True)
        return None
    theta, meta = load_proposer(path)
    tau = meta.get("thresholds", {}).get("%dx%d" % (w, h))
    if tau is None:
        return None
    wb = torch.from_numpy(theta).cuda().to(torch.bfloat16).view(torch.int16).contiguous()
    fe.run()
    exact = keypoint_sets(fe)
    fe.run_learned(wb, tau)
    got = keypoint_sets(fe)
    kept = float(fe.cell_mask.float().mean().item())
    ref_n = sum(len(r) for r in exact)
    hit = sum(len(r & g) for r, g in zip(exact, got))
    g2 = fe.capture(fe.run_learned, params_bf16=wb, thresh=tau)
    for _ in range(args.warmup):
        g2.replay()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        g2.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    c, b = fe.ctx, fe.batch
    calls = {
        "cnn_propose": lambda: vsfe.cnn_propose(c, b, fe.pyr, wb, tau, fe.cnn_ws, fe.grid_logits, fe.cell_logits,
                                                fe.cell_mask, fe.status, stream),
        "fast_br_detect_gated": lambda: vsfe.fast_br_detect(c, b, fe.images, fe.pyr, fe.cell_mask, fe.cell_keys,
                                                            None, fe.status, stream),
    }
    ones = torch.ones_like(fe.cell_mask)
    calls["fast_br_detect_all_cells_kept"] = lambda: vsfe.fast_br_detect(c, b, fe.images, fe.pyr, ones, fe.cell_keys,
                                                                         None, fe.status, stream)
    ideal, ideal_res = ideal_gate(args, fe, sizes, stream, exact, exact_value)
    calls["fast_br_detect_ideal_mask"] = lambda: vsfe.fast_br_detect(c, b, fe.images, fe.pyr, ideal, fe.cell_keys,
                                                                     None, fe.status, stream)
    call_us = {k: round(time_call(f, args.kernel_reps, stream), 2) for k, f in calls.items()}
    value = (len(sizes) // 2) * 1000.0 / ms
    return {"value": round(value, 1), "unit": "stereo pairs/s", "ms_per_step": round(ms, 4),
            "speedup_vs_exact": round(value / exact_value, 4), "recall": round(hit / max(ref_n, 1), 5),
            "precision": round(hit / max(sum(len(g) for g in got), 1), 5), "kept_cell_frac": round(kept, 4),
            "thresh": tau, "weights": os.path.relpath(path, ROOT), "calls_us": call_us,
            "ideal_gate": ideal_res}


def ideal_gate(args, fe, sizes, stream, exact, exact_value):
    """The gate's ceiling on this batch: the path gated by exactly the
    native-scale cells that hold a final keypoint of the exact path (what a
    proposer with perfect recall would keep at the smallest kept fraction),
    with no proposer at all.  Returns the mask and the timed result."""
    import torch
    from paper_2410_04090_amd import labels
    torch.cuda.synchronize()
    fe.run()
    counts = fe.kp_count.cpu().numpy()
    n_max = fe.params.n_max
    x0 = fe.kps["x0"].cpu().numpy().view(np.uint16)
    y0 = fe.kps["y0"].cpu().numpy().view(np.uint16)
    parts = []
    for i, (w, h) in enumerate(sizes):
        s = slice(i * n_max, i * n_max + int(counts[i]))
        parts.append(labels.positive_cells(x0[s], y0[s], w, h).reshape(-1))
    mask = np.concatenate(parts).astype(np.uint8)
    if mask.size != fe.cell_mask.numel():
        raise RuntimeError("native-scale cell count %d differs from the batch's %d" % (mask.size, fe.cell_mask.numel()))
    ideal = torch.from_numpy(mask).to(fe.cell_mask.device)
    fe.run(mask=ideal)
    got = keypoint_sets(fe)
    ref_n = sum(len(r) for r in exact)
    hit = sum(len(r & g) for r, g in zip(exact, got))
    g3 = fe.capture(fe.run, mask=ideal)
    for _ in range(args.warmup):
        g3.replay()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        g3.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    value = (len(sizes) // 2) * 1000.0 / ms
    return ideal, {"what": "gated by the cells holding a final keypoint of the exact path, no proposer",
                   "value": round(value, 1), "ms_per_step": round(ms, 4),
                   "speedup_vs_exact": round(value / exact_value, 4), "recall": round(hit / max(ref_n, 1), 5),
                   "kept_cell_frac": round(float(mask.mean()), 4)}


def middle_end(args, fe, stream):
    """Per-call times of the middle-end steps after stereo matching: sub-pixel
    refinement of the matches, and descriptor matching of every image's
    keypoints against a reference set (here the image's own keypoints, whose
    windows hold the same candidates a previous frame's would)."""
    import torch
    from paper_2410_04090_amd import vsfe
    c, b = fe.ctx, fe.batch
    fe.refine(stream=stream)
    torch.cuda.synchronize()
    n_left = int(sum(fe.kp_count[0::2].tolist()))
    refined = sum(int((fe.refined(p)[0] != -(2 ** 31)).sum()) for p in range(fe.n // 2))
    ws = torch.zeros(max(vsfe.feature_match_workspace(b), 4), dtype=torch.uint8, device="cuda")
    cap = int(fe.info.kp_capacity)
    idx = torch.zeros(cap, dtype=torch.int32, device="cuda")
    d1 = torch.zeros(cap, dtype=torch.int16, device="cuda")
    d2 = torch.zeros(cap, dtype=torch.int16, device="cuda")
    calls = {
        "stereo_refine": lambda: fe.refine(stream=stream),
        "feature_match": lambda: vsfe.feature_match(c, b, fe.kps, fe.kp_count, fe.desc, fe.kps, fe.kp_count, fe.desc,
                                                    16, 1, 64, 90, ws, idx, d1, d2, fe.status, stream),
    }
    out = {k: round(time_call(f, args.kernel_reps, stream), 2) for k, f in calls.items()}
    return {"calls_us": out, "refined_frac": round(refined / max(n_left, 1), 4),
            "refine_window": 2 * fe.REFINE_HALF_WINDOW + 1, "refine_radius": fe.REFINE_RADIUS,
            "feature_match": {"radius": 16, "level_band": 1, "match_th": 64, "ratio_pct": 90}}


def culling_ablation(args, wl, fe, stream):
    """Feature Culling over a materialised response matrix with the paper's
    thread schemes (MLPT + TEWA, log2 reduction, MLPT with one block per
    cell) against the fused culling of the detector: per level of this
    batch at its cell sizes, and at level 0 with the paper's cell sizes."""
    import torch
    from paper_2410_04090_amd import vsfe
    c, b = fe.ctx, fe.batch
    crf = torch.zeros(max(int(fe.info.crf_elems), 1), dtype=torch.int16, device="cuda")
    # the keys of the largest (level, cell) queried: n_images x its stride
    cells = [(lv, int(fe.level_info(0, lv).cell)) for lv in range(wl.params.n_levels)]
    cells += [(0, cell) for cell in (23, 17, 13, 7, 3)]
    n_keys = max(fe.n * vsfe.fc_cull_stride(b, lv, cell) for lv, cell in cells)
    keys = torch.zeros(max(n_keys, 1), dtype=torch.int32, device="cuda")
    fused = time_call(lambda: vsfe.fast_br_detect(c, b, fe.images, fe.pyr, None, fe.cell_keys, None, fe.status,
                                                  stream), args.kernel_reps, stream)
    dump = time_call(lambda: vsfe.fast_br_detect(c, b, fe.images, fe.pyr, None, fe.cell_keys, crf, fe.status,
                                                 stream), args.kernel_reps, stream)
    schemes = {"mlpt_tewa": 0, "log2_block_per_cell": 1, "mlpt_block_per_cell": 2}
    per_level = []
    for lv in range(wl.params.n_levels):
        cell = int(fe.level_info(0, lv).cell)
        n_loc = max(1, -(-cell // 8))
        row = {"level": lv, "cell": cell}
        for name, sc in schemes.items():
            row[name] = round(time_call(lambda: vsfe.fc_cull_crf(c, b, crf, lv, cell, sc, n_loc, keys, fe.status,
                                                                 stream), args.kernel_reps, stream), 2)
        per_level.append(row)
    sweep = []
    for cell in (23, 17, 13, 7, 3):
        n_loc = max(1, -(-cell // 8))
        row = {"cell": cell}
        for name, sc in schemes.items():
            row[name] = round(time_call(lambda: vsfe.fc_cull_crf(c, b, crf, 0, cell, sc, n_loc, keys, fe.status,
                                                                 stream), args.kernel_reps, stream), 2)
        sweep.append(row)
    return {"fused_detect_us": round(fused, 2), "detect_with_dump_us": round(dump, 2), "per_level_us": per_level,
            "level0_cell_sweep_us": sweep, "images": fe.n}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch64_1080p", choices=["pair_1241x376", "batch32_mixed", "batch64_1080p"])
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-procs", type=int, default=1,
                    help="processes for the oracle baseline (default 1: single-threaded)")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--procs", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the middle-end calls, the culling ablation and the repeatability harness")
    ap.add_argument("--proposer", default=None, help="proposer weights (default: the packaged ones for the image size)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--probe", action="store_true",
                    help="only measure the VALU issue rate and LDS bandwidth ceilings and exit")
    args = ap.parse_args()
    if args.probe:
        ceiling_probe()
        return
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py: one GPU only (--gpus 1); stereo pairs are independent, so a batch would "
              "shard across GPUs by whole pairs, each GPU replaying its own graph", file=sys.stderr)
        sys.exit(2)

    from synth import configs, pattern as pat
    wl = configs.WORKLOADS[args.workload]()
    pattern = pat.brief_pattern()
    t_gen = time.perf_counter()
    imgs = make_images(wl, args.procs)
    t_gen = time.perf_counter() - t_gen
    print("generated %d images in %.1f s" % (len(imgs), t_gen), file=sys.stderr, flush=True)
    # the oracle baseline runs before this process touches the GPU (its
    # worker processes are forked from a process without a device context)
    cpu = None if args.no_cpu else cpu_baseline(wl, imgs, pattern, args.cpu_budget, args.cpu_procs)

    import torch
    from paper_2410_04090_amd import vsfe
    from paper_2410_04090_amd.frontend import Frontend
    torch.cuda.set_device(0)
    sizes = wl.image_sizes()
    fe = Frontend(wl.params, sizes, pattern)
    fe.upload(imgs)
    torch.cuda.synchronize()
    fe.run()
    torch.cuda.synchronize()
    assert int(fe.status.item()) == 0, "device status flagged"
    print("first run ok", file=sys.stderr, flush=True)

    tune = None
    if not args.no_autotune:
        tune = fe.autotune(reps=3)
        print("autotuned tiles w=%s h=%s" % (tune["tile_w"], tune["tile_h"]), file=sys.stderr, flush=True)

    # ---- timed region: K graph replays of the whole exact path
    g = fe.capture()
    for _ in range(args.warmup):
        fe.replay()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        g.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    n_pairs = len(sizes) // 2
    value = n_pairs * args.steps / (gpu_ms / 1000.0)
    print("timed %d steps: %.3f ms/step (wall %.3f s)" % (args.steps, ms_per_step, wall), file=sys.stderr,
          flush=True)

    # ---- per-call durations (HIP events on the launching stream)
    c, b = fe.ctx, fe.batch
    reps = args.kernel_reps
    calls = {
        "pyramid_build": lambda: vsfe.pyramid_build(c, b, fe.images, fe.pyr, fe.status, stream),
        "fast_br_detect": lambda: vsfe.fast_br_detect(c, b, fe.images, fe.pyr, None, fe.cell_keys, None,
                                                      fe.status, stream),
        "pyca_cull_aggregate": lambda: vsfe.pyca_cull_aggregate(c, b, fe.cell_keys, fe.workspace, fe.kps,
                                                                fe.kp_count, fe.status, stream),
        "orb_describe": lambda: vsfe.orb_describe(c, b, fe.images, fe.pyr, fe.kps, fe.kp_count, fe.desc,
                                                  fe.status, stream),
        "stereo_match": lambda: vsfe.stereo_match(c, b, fe.kps, fe.kp_count, fe.desc, fe.match_idx,
                                                  fe.match_dist, fe.match_disp, fe.status, stream),
    }
    call_us = {k: time_call(f, reps, stream) for k, f in calls.items()}
    torch.cuda.synchronize()

    # ---- algorithmic bytes per call, whole batch: what each call must read and write
    L = wl.params.n_levels
    px_all = px_up = px_last = sum_l0 = 0
    n_cells = int(fe.info.n_cells)
    for (w, h) in sizes:
        ls = level_sizes(w, h, L)
        px_all += sum(a * bb for a, bb in ls)
        px_up += sum(a * bb for a, bb in ls[1:])
        px_last += ls[-1][0] * ls[-1][1]
        sum_l0 += w * h
    n_kp = int(fe.kp_count.sum().item())
    n_left = int(sum(fe.kp_count[0::2].tolist()))
    alg = {
        # launch l reads level l-1 and writes level l
        "pyramid_build": (px_all - px_last) + px_up,
        # read every level pixel once, write one key per cell
        "fast_br_detect": px_all + 4 * n_cells,
        # keys in, ranks out and back, keypoints out (16 B each)
        "pyca_cull_aggregate": 4 * n_cells * 4 + 16 * n_kp,
        # per keypoint: its 37x37 neighbourhood, 16 B of keypoint in, 32 B + 1 B out
        "orb_describe": n_kp * (37 * 37 + 16 + 33),
        # per left keypoint: its record + descriptor in, 8 B of match out
        "stereo_match": n_left * (48 + 8),
    }
    dominant = max(call_us, key=call_us.get)
    ach = alg[dominant] / (call_us[dominant] * 1e-6) / 1e9
    traffic = stored_traffic(dominant, args.workload)
    hbm = {"achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
           "traffic": traffic, "alg_bytes_per_launch": int(alg[dominant])}
    sq = stored_counters(dominant, args.workload)
    valu = None
    if sq is not None:
        # issued VALU instructions over the launch against the issue peak
        issue = sq["insts_valu_per_launch"] / (call_us[dominant] * 1e-6) / VALU_WAVE_INSTS_PER_S
        valu = {"achieved": round(sq["insts_valu_per_launch"] * 64 / (call_us[dominant] * 1e-6) / 1e12, 2),
                "peak": round(VALU_LANE_OPS_PEAK_T, 1), "unit": "T lane-ops/s (issued int32 VALU)",
                "frac": round(issue, 4), "insts_valu_per_launch": sq["insts_valu_per_launch"],
                "insts_salu_per_launch": sq["insts_salu_per_launch"]}
        ceil = stored_ceiling()
        if ceil is not None:
            # the same issue rate against what the probe kernel reaches on this chip
            valu["measured_ceiling_wave_insts_per_s"] = ceil
            valu["frac_of_measured_ceiling"] = round(sq["insts_valu_per_launch"] / (call_us[dominant] * 1e-6) / ceil, 4)
    if valu is not None and valu["frac"] > hbm["frac"]:
        roof = {"kernel": dominant, "bound": "alu", "achieved": valu["achieved"], "peak": valu["peak"],
                "unit": valu["unit"], "frac": valu["frac"], "traffic": traffic, "hbm": hbm, "valu": valu}
    else:
        roof = {"kernel": dominant, "bound": "hbm", "achieved": hbm["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm["frac"], "traffic": traffic, "hbm": hbm, "valu": valu}
    roof.update({"avg_launch_us": round(call_us[dominant], 2), "source_sha": source_sha(dominant)})
    # whole-path algorithmic bytes: level 0 read once, every other level
    # written once and read once, keypoints (16 B) and descriptors (32 B)
    # written, matches (8 B per left keypoint) written
    path_bytes = sum_l0 + 2 * px_up + 48 * n_kp + 8 * n_left
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "stereo pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wl.name, "pairs": n_pairs, "sizes": sorted(set("%dx%d" % s for s in sizes)),
                   "levels": L, "n_max": wl.params.n_max, "path": "exact"},
        "roofline": roof,
        "calls_us": {k: round(v, 2) for k, v in call_us.items()},
        "path_alg_bytes": int(path_bytes),
        "path_hbm_frac": round(path_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "calls_alg_bytes": int(sum(alg.values())),
        "keypoints_per_image": round(n_kp / len(sizes), 1),
        "fast_br_grid_threads": int(vsfe.batch_info(fe.batch).n_det_items) * 256,
    }
    if tune is not None:
        res["autotune"] = tune
    if not args.no_extras and fe.stereo:
        res["middle_end"] = middle_end(args, fe, stream)
    learned = None if args.no_learned else learned_path(args, fe, sizes, stream, value)
    if learned is not None:
        res["learned"] = learned
    if not args.no_extras:
        res["culling_ablation"] = culling_ablation(args, wl, fe, stream)
    fe.close()
    if not args.no_extras:
        from paper_2410_04090_amd import repeatability
        t_rep = time.perf_counter()
        rep = repeatability.run()
        res["repeatability"] = {"mean_f1": {k: round(v, 4) for k, v in rep["mean_f1"].items()},
                                "f1_per_angle": {str(a): {k: round(v["f1"], 4) for k, v in rep["per_angle"][a].items()}
                                                 for a in rep["per_angle"]},
                                "scenes": rep["scenes"], "size": rep["size"], "eps": rep["eps"],
                                "tol_px": rep["tol_px"], "seconds": round(time.perf_counter() - t_rep, 1)}
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
