"""Benchmark of the rasterizer hot path on one MI355X.

One step = one pass of the whole path on the room workload: anchor decode
(40k anchors x 10 offsets = 400k Gaussians, ~300k in view), forward render of a
1200x680 view (projection, binning, depth and tile sorts, compositing), L1
colour + 0.5 L1 depth loss against a target rendered once at a pose perturbed by
2 cm / 1 degree, the replayed backward to the Gaussians and the SE(3) pose, and
the decode backward to features, MLP weights, offsets and scalings.  Inputs are
synthetic, seeded and resident in HBM before timing starts.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline]

Prints one JSON line: Mpix/s of forward+backward, the roofline of the stage
that takes the most time (measured with HIP events on the library's stream
during the timed steps), and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak
FP32_MFMA_PEAK_TFLOPS = 157.3

# Algorithmic work per evaluated (pixel, list entry), the exponential and the
# division counted as one flop each: the forward about 25 flops plus the
# exponential, the adjoint about 70 flops plus the exponential and the division.
FLOP_EVAL_FWD = 26
FLOP_EVAL_BWD = 72


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--stages", action="store_true", help="also print a per-stage table to stderr")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--no-ba", action="store_true", help="skip the 12-keyframe bundle-adjustment window")
    ap.add_argument("--ba-steps", type=int, default=10)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving replay")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per arrival rate")
    ap.add_argument("--serve-qps", type=str, default="50,100,200,400,1000,2000,4000")
    ap.add_argument("--only", choices=("main", "ba", "ba_view", "serve", "view", "mask", "codebook", "rvq", "track"),
                    default=None,
                    help="run one section only (for profiling)")
    return ap.parse_args()


def room_inputs():
    from paper_2403_11247_amd import scenes
    a = scenes.room_anchors(40000, k=10)
    m = scenes.room_mlp()
    cam, pose = scenes.room_camera()
    tpose = scenes.perturb_pose(pose, 2)
    return a, m, cam, pose, tpose


def stage_bytes(stage, n, nvis, P, na, W, H, tiles=0):
    """Algorithmic HBM bytes of one launch of a stage."""
    if stage == "decode":
        return na * (12 + 128 + 12 + 120) + n * 56
    if stage == "preprocess":
        return n * (56 + 16) + nvis * 48
    if stage == "depth_sort":
        # histogram read, first pass reads all keys and writes the kept (key, index),
        # three more passes read and write 8 B per kept item
        return n * 4 + n * 4 + nvis * 8 + 3 * nvis * 16
    if stage == "tile_sort":
        passes = max(1, (max(int(tiles) - 1, 1).bit_length() + 7) // 8)
        return P * 4 + passes * P * 16
    if stage == "emit":
        return nvis * 28 + P * 8
    if stage == "preprocess_bwd":
        return nvis * (40 + 40 + 56) + n * 4
    if stage == "decode_bwd":
        return na * (272 + 272) + n * 56
    return None


KERNEL_SOURCES = {"composite": "render.hip", "composite_bwd": "render.hip", "decode": "decode.hip",
                  "decode_bwd": "decode.hip", "preprocess": "preprocess.hip", "preprocess_bwd": "preprocess.hip",
                  "depth_sort": "sort.hip", "tile_sort": "sort.hip", "emit": "binning.hip"}


def measured_traffic(stage):
    """HBM bytes per launch of `stage` from the committed counter summary, or
    None when there is none or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or stage not in KERNEL_SOURCES:
        return None
    with open(path) as f:
        rec = json.load(f).get(stage)
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2403_11247_amd", "csrc", KERNEL_SOURCES[stage])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec.get("source_sha256"):
            return None
    return int(rec["bytes_per_launch"])


def cpu_baseline_run(budget_s):
    """The oracle, as it stands, on the same workload: full fwd+bwd steps until
    the time budget is used (at least one, at most three).  The oracle's
    OpenMP loops use OMP_NUM_THREADS threads; its adjoint is single-threaded."""
    from oracle import decode as odec, raster
    from paper_2403_11247_amd import scenes
    a, m, cam, pose, tpose = room_inputs()
    dec = odec.decode(a, m)
    g = scenes.Gaussians(*[dec[f].astype(np.float32) for f in ("mean", "scale", "quat", "opacity", "color")])
    tgt = raster.render(g, cam, tpose)
    steps = 0
    t0 = time.perf_counter()
    while True:
        d = odec.decode(a, m)
        gg = scenes.Gaussians(*[d[f].astype(np.float32) for f in ("mean", "scale", "quat", "opacity", "color")])
        r = raster.render(gg, cam, pose)
        npix = cam.width * cam.height
        dc = np.sign(r["color"] - tgt["color"]) / npix
        dd = 0.5 * np.sign(r["depth"] - tgt["depth"]) / npix
        gr = raster.render_backward(gg, cam, pose, r, dc, dd, np.zeros_like(dd))
        odec.decode_backward(a, m, d, gr)
        steps += 1
        if time.perf_counter() - t0 >= budget_s or steps >= 3:
            break
    dt = (time.perf_counter() - t0) / steps
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(cam.width * cam.height / dt / 1e6, 4), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle", "step_s": round(dt, 3),
            "sample": f"{steps} full fwd+bwd step(s) of the room workload (1200x680, 400k Gaussians), "
                      f"{dt:.2f} s each; projection/compositing forward on {threads} OpenMP thread(s), "
                      f"adjoint single-threaded"}


def cpu_baseline(budget_s):
    """The oracle timed twice, each in a child process of its own (the thread
    count of its OpenMP loops is fixed when a process starts): on all the host
    threads this process may use, and on one thread."""
    import subprocess
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    runs = {}
    for n in (cores, 1):
        env = dict(os.environ, OMP_NUM_THREADS=str(n))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                            "--cpu-budget-s", str(budget_s)], env=env, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("CPU baseline run failed:\n" + r.stderr[-2000:])
        runs[n] = json.loads(r.stdout.strip().splitlines()[-1])
    out = dict(runs[cores])
    out["single_thread"] = {k: runs[1][k] for k in ("value", "unit", "cores", "step_s")}
    return out


F = ("mean", "scale", "quat", "opacity", "color")


def _up(x, dev, dt=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).to(dev, dt or torch.float32)


def _decoded_map(n_anchors, spacing, seed, dev):
    """Room map decoded on the GPU (anchor decode kernel)."""
    from paper_2403_11247_amd import scenes
    from paper_2403_11247_amd.vcgs import decode_anchors
    a = scenes.room_anchors(n_anchors, k=10, spacing=spacing, seed=seed)
    m = scenes.room_mlp(seed=seed)
    A = [_up(x, dev) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    G = decode_anchors(*A)
    return [G[f] for f in F]


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def ba_section(args, dev):
    """12 keyframes (4 x 320x240, 4 x 640x480, 4 x 1200x680) of a 500k-Gaussian
    room, forward + L1 loss + backward to the Gaussians and the 12 poses: the
    plain per-view loop against one batched pass, eager and as a replayed
    hipGraph, with the compositing configuration chosen by the autotuner."""
    import torch
    from paper_2403_11247_amd import autotune, scenes, vcgs
    gd = _decoded_map(50000, 0.05, 1, dev)
    n = int(gd[3].shape[0])
    cams, poses = scenes.ba_window(12)
    tposes = [scenes.perturb_pose(p, 100 + i) for i, p in enumerate(poses)]
    targets = []
    for c, p in zip(cams, tposes):
        C, D, _, _ = vcgs.render_forward(*gd, c, p, keep_state=False)
        targets.append((C, D))
    acc = {k: torch.zeros_like(t) for k, t in zip(F, gd)}
    dposes = torch.empty((len(cams), 6), device=dev)

    def plain():
        for t in acc.values():
            t.zero_()
        for i, (c, p, tg) in enumerate(zip(cams, poses, targets)):
            C, D, _, st = vcgs.render_forward(*gd, c, p)
            _, dlc, dld = vcgs.l1_loss(C, D, tg[0], tg[1], 0.5)
            gr, dp = vcgs.render_backward(st, *gd, c, p, dlc, dld, None)
            for k in F:
                acc[k].add_(gr[k])
            dposes[i].copy_(dp)
            st.free()

    saved = autotune.current()
    eager = vcgs.BatchWindow(n, cams, backward=True)
    best, table = autotune.tune(eager, (*gd, poses, targets), reps=3)
    graph = vcgs.BatchWindow(n, cams, backward=True, graph=True)
    # the plain loop without its per-view pair-count synchronisations: one
    # single-view pass per keyframe, each with buffers sized once
    singles = [vcgs.BatchWindow(n, [c], backward=True) for c in cams]

    def plain_nosync():
        for i, (w, p, tg) in enumerate(zip(singles, poses, targets)):
            w.run(*gd, [p], [tg], check=False)
            if i == 0:
                for k in F:
                    acc[k].copy_(w.grads[k])
            else:
                for k in F:
                    acc[k].add_(w.grads[k])
            dposes[i].copy_(w.dpose[0])

    def timed_nosync(fn, windows):
        for w, p, tg in windows:  # size every plan (one synchronising run each)
            w.run(*gd, p, tg)
        ms = _timed(fn, args.ba_steps, 2)
        for w, p, tg in windows:  # the timed passes fitted their buffers
            w.run(*gd, p, tg)
            assert w.check(), "a timed pass outgrew its pair buffers"
        return ms

    ms_plain = _timed(plain, args.ba_steps, 2)
    ms_plain_nosync = timed_nosync(plain_nosync, [(w, [p], [tg]) for w, p, tg in zip(singles, poses, targets)])
    ms_eager = timed_nosync(lambda: eager.run(*gd, poses, targets, check=False), [(eager, poses, targets)])
    ms_graph = timed_nosync(lambda: graph.run(*gd, poses, targets, check=False), [(graph, poses, targets)])
    # accuracy of the batched pass against the plain loop (same inputs)
    plain()
    graph.run(*gd, poses, targets)
    torch.cuda.synchronize()

    def rel(a, b):
        return float((a - b).abs().max() / b.abs().max().clamp_min(1e-30))

    g_err = max(rel(graph.grads[k], acc[k]) for k in F)
    p_err = rel(graph.dpose, dposes)
    worst = max(table, key=lambda kv: kv[1])[1] if table else None
    autotune.apply(saved)
    pix = sum(int(c.width) * int(c.height) for c in cams)
    return {"workload": "room 50k anchors x 10 (500k Gaussians), 12 keyframes 4x320x240 + 4x640x480 + 4x1200x680 "
                        "on a 1.5 m circle, fwd + L1 loss + bwd to Gaussians and 12 poses",
            "gaussians": n, "pixels": pix, "pairs": graph.pairs,
            "plain_ms": round(ms_plain, 3), "plain_nosync_ms": round(ms_plain_nosync, 3),
            "batch_eager_ms": round(ms_eager, 3), "batch_graph_ms": round(ms_graph, 3),
            "speedup_graph_vs_plain": round(ms_plain / ms_graph, 2),
            "speedup_graph_vs_plain_nosync": round(ms_plain_nosync / ms_graph, 2),
            "speedup_eager_vs_plain": round(ms_plain / ms_eager, 2),
            "timing": "batched passes and the no-sync loop run back to back without host synchronisation; "
                      "one check after the timed passes confirms no pass outgrew its pair buffers",
            "batch_graph_mpix_s": round(pix / (ms_graph * 1e-3) / 1e6, 1),
            "grad_rel_err_vs_plain": g_err, "pose_grad_rel_err_vs_plain": p_err,
            "autotune": {"best": best, "candidates": len(table),
                         "best_ms": round(min(t for _, t in table) * 1e3, 3) if table else None,
                         "worst_ms": round(worst * 1e3, 3) if worst else None}}


def ba_view_section(args, dev):
    """The BA window with the view-dependent decode (eqs. (8)-(9)): the 12
    keyframes decode their own 500k-Gaussian sets from the same anchors and MLP
    in one launch (into the stacked per-view set), one batched forward + L1 +
    backward pass over the stacked sets (per-view mode, replayed hipGraph), and
    one decode backward that sums the anchor and MLP gradients over the window
    and gives each keyframe's camera-centre gradient; against the plain loop of
    decode, render, loss, backward and decode backward per keyframe."""
    import torch
    from paper_2403_11247_amd import scenes, vcgs
    a = scenes.room_anchors(50000, k=10, spacing=0.05, seed=1)
    m = scenes.room_mlp_view(seed=1)
    A = [_up(x, dev) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    n = a.xa.shape[1] * 10
    cams, poses = scenes.ba_window(12)
    V = len(cams)
    centres = np.stack([vcgs.camera_centre(p) for p in poses])
    targets = []
    for c, p in zip(cams, poses):
        tp = scenes.perturb_pose(p, 200 + len(targets))
        G = vcgs.decode_anchors(*A, cam_centre=vcgs.camera_centre(tp))
        C, D, _, _ = vcgs.render_forward(*[G[f] for f in F], c, tp, keep_state=False)
        targets.append((C, D))
    stacked = vcgs.decode_anchors_views(*A, centres)
    win = vcgs.BatchWindow(n, cams, backward=True, graph=True, per_view=True)
    got = {}

    def batched():
        vcgs.decode_anchors_views(*A, centres, out=stacked)
        win.run(*[stacked[f] for f in F], poses, targets)
        ag = vcgs.decode_anchors_views_backward(*A, win.grads, centres)
        got["dpose"] = vcgs.add_centre_pose_grad(poses, ag["cam"], win.dpose)
        got["W1"] = ag["W1"]

    ref = {"dpose": torch.empty((V, 6), device=dev)}

    def plain():
        dW1 = None
        for v, (c, p, tg) in enumerate(zip(cams, poses, targets)):
            G = vcgs.decode_anchors(*A, cam_centre=centres[v])
            gs = [G[f] for f in F]
            C, D, _, st = vcgs.render_forward(*gs, c, p)
            _, dlc, dld = vcgs.l1_loss(C, D, tg[0], tg[1], 0.5)
            gr, dp = vcgs.render_backward(st, *gs, c, p, dlc, dld, None)
            ag = vcgs.decode_anchors_backward(*A, gr, cam_centre=centres[v])
            vcgs.add_centre_pose_grad([p], ag["cam"].reshape(1, 3), dp.reshape(1, 6))
            ref["dpose"][v].copy_(dp)
            dW1 = ag["W1"] if dW1 is None else dW1 + ag["W1"]
            st.free()
        ref["W1"] = dW1

    ms_plain = _timed(plain, args.ba_steps, 2)
    ms_batch = _timed(batched, args.ba_steps, 2)
    plain()
    batched()
    torch.cuda.synchronize()

    def rel(x, y):
        return float((x - y).abs().max() / y.abs().max().clamp_min(1e-30))

    pix = sum(int(c.width) * int(c.height) for c in cams)
    return {"workload": "room 50k anchors x 10 with the view-dependent decode, 12 keyframes 4x320x240 + "
                        "4x640x480 + 4x1200x680: decode of the 12 views, fwd + L1 + bwd, decode bwd summed over "
                        "the window, pose gradients through render and decode",
            "gaussians_per_view": n, "pixels": pix,
            "plain_ms": round(ms_plain, 3), "batch_graph_ms": round(ms_batch, 3),
            "speedup_vs_plain": round(ms_plain / ms_batch, 2),
            "pose_grad_rel_err_vs_plain": rel(got["dpose"], ref["dpose"]),
            "mlp_grad_rel_err_vs_plain": rel(got["W1"], ref["W1"])}


def view_decode_section(args, dev, steps=20, warmup=5):
    """The room step with the view-dependent decode (eqs. (8)-(9)): the MLP
    input is [f_a, delta, d] from the camera centre, so the decode runs per view
    and its backward adds the camera-centre path to the pose gradient."""
    import torch
    from paper_2403_11247_amd import scenes, vcgs
    a = scenes.room_anchors(40000, k=10)
    m = scenes.room_mlp_view(seed=0)
    cam, pose = scenes.room_camera()
    tpose = scenes.perturb_pose(pose, 2)
    A = [_up(x, dev) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    c_now, c_tgt = vcgs.camera_centre(pose), vcgs.camera_centre(tpose)
    G0 = vcgs.decode_anchors(*A, cam_centre=c_tgt)
    tC, tD, _, _ = vcgs.render_forward(*[G0[f] for f in F], cam, tpose, keep_state=False)

    def step():
        G = vcgs.decode_anchors(*A, cam_centre=c_now)
        C, D, _, st = vcgs.render_forward(*[G[f] for f in F], cam, pose)
        _, dlc, dld = vcgs.l1_loss(C, D, tC, tD, 0.5)
        grads, dpose = vcgs.render_backward(st, *[G[f] for f in F], cam, pose, dlc, dld, None)
        ag = vcgs.decode_anchors_backward(*A, grads, cam_centre=c_now)
        st.free()
        return vcgs.add_centre_pose_grad([pose], ag["cam"].reshape(1, 3), dpose.reshape(1, 6))

    ms = _timed(step, steps, warmup)
    return {"workload": "room step with the view-dependent decode (36-d MLP input), pose gradient through "
                        "render and decode", "ms_per_step": round(ms, 4),
            "mpix_s": round(cam.width * cam.height / (ms * 1e-3) / 1e6, 2)}


def mask_step_section(args, dev, steps=20, warmup=5, lam=5e-4):
    """The room step with the mask training of eq. (13): decode with the mask,
    forward with per-Gaussian hit counts, L1 loss, backward, the mask loss over
    the view frustum added to the decode's mask gradient; and the pruning that
    ends a window (mask and hit counts), timed on its own."""
    import torch
    from paper_2403_11247_amd import scenes, vcgs
    a = scenes.room_anchors(40000, k=10)
    m = scenes.room_mlp(seed=0)
    n = a.xa.shape[1] * 10
    mask, _, _ = scenes.mask_and_codebook(n)
    cam, pose = scenes.room_camera()
    tpose = scenes.perturb_pose(pose, 2)
    A = [_up(x, dev) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    ml = _up(mask, dev)
    G0 = vcgs.decode_anchors(*A, mask_logit=ml)
    tC, tD, _, _ = vcgs.render_forward(*[G0[f] for f in F], cam, tpose, keep_state=False)
    hits = torch.zeros(n, dtype=torch.int32, device=dev)

    def step():
        G = vcgs.decode_anchors(*A, mask_logit=ml)
        C, D, _, st = vcgs.render_forward(*[G[f] for f in F], cam, pose, hits=hits)
        _, dlc, dld = vcgs.l1_loss(C, D, tC, tD, 0.5)
        grads, dpose = vcgs.render_backward(st, *[G[f] for f in F], cam, pose, dlc, dld, None)
        ag = vcgs.decode_anchors_backward(*A, grads, mask_logit=ml)
        lm, _ = vcgs.mask_loss(ml, st.tile_count(), lam, dl_dm=ag["mask_logit"])
        st.free()
        return dpose, ag, lm

    ms = _timed(step, steps, warmup)
    ms_prune = _timed(lambda: vcgs.mask_prune(ml, hits, 0.01, 1), steps, warmup)
    keep, idx = vcgs.mask_prune(ml, hits, 0.01, 1)
    return {"workload": "room step with the mask training of eq. (13) (hit counts, frustum mask loss) and the "
                        "window-end pruning, 400k Gaussians, 1200x680",
            "ms_per_step": round(ms, 4), "mpix_s": round(cam.width * cam.height / (ms * 1e-3) / 1e6, 2),
            "prune_ms": round(ms_prune, 4), "kept": int(idx.numel()), "n": n}


def codebook_section(args, dev, steps=20, warmup=5):
    """The compacted room (mask + residual codebooks, Sec. 3.3-3.4): 2-stage
    residual k-means codebooks of 4096 x 7 fit to the room's decoded
    (log-scale, quaternion), mask logits N(2, 1); the render against the
    unquantized one (PSNR), and the room step with codebook and mask gradients."""
    import torch
    from paper_2403_11247_amd import codebook_fit, scenes, vcgs
    a = scenes.room_anchors(40000, k=10)
    m = scenes.room_mlp(seed=0)
    n = a.xa.shape[1] * 10
    cam, pose = scenes.room_camera()
    tpose = scenes.perturb_pose(pose, 2)
    A = [_up(x, dev) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    G0 = vcgs.decode_anchors(*A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    books, idx = codebook_fit.residual_kmeans(codebook_fit.shape_vectors(G0), stages=2, size=4096, iters=10)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    mask, _, _ = scenes.mask_and_codebook(n)
    ml = _up(mask, dev)
    kw = dict(books=books, idx=idx, mask_logit=ml)
    Gq = vcgs.decode_anchors(*A, **kw)
    C0, D0, _, _ = vcgs.render_forward(*[G0[f] for f in F], cam, pose, keep_state=False)
    Cq, Dq, _, _ = vcgs.render_forward(*[Gq[f] for f in F], cam, pose, keep_state=False)
    tC, tD, _, _ = vcgs.render_forward(*[Gq[f] for f in F], cam, tpose, keep_state=False)
    torch.cuda.synchronize()
    psnr = codebook_fit.psnr(Cq.clamp(0, 1), C0.clamp(0, 1))
    depth_mae = float((Dq - D0).abs().mean())

    def step():
        G = vcgs.decode_anchors(*A, **kw)
        C, D, _, st = vcgs.render_forward(*[G[f] for f in F], cam, pose)
        _, dlc, dld = vcgs.l1_loss(C, D, tC, tD, 0.5)
        grads, dpose = vcgs.render_backward(st, *[G[f] for f in F], cam, pose, dlc, dld, None)
        ag = vcgs.decode_anchors_backward(*A, grads, **kw)
        st.free()
        return dpose, ag

    ms = _timed(step, steps, warmup)
    return {"workload": "room 40k anchors x 10 with mask logits N(2,1) and 2-stage residual k-means codebooks "
                        "4096 x 7 (10 Lloyd iterations) for log-scale and rotation; fwd + L1 + bwd incl. codebook "
                        "(straight-through) and mask gradients, 1200x680",
            "ms_per_step": round(ms, 4), "mpix_s": round(cam.width * cam.height / (ms * 1e-3) / 1e6, 2),
            "psnr_vs_unquantized_db": round(psnr, 2), "depth_mae_m": round(depth_mae, 5),
            "codebook_fit_s": round(fit_s, 2), "gaussians": n}


def rvq_section(args, dev, steps=50, warmup=5):
    """Residual vector quantization (eqs. (14)-(15)) of the room map's
    attributes: assignment, reconstruction, loss and code gradient in one call.
    Algorithmic work: n * L * P * 2D flops of distance (the compare and select
    per code are not counted), priced against the FP32 vector peak."""
    import torch
    from paper_2403_11247_amd import scenes, vcgs
    rows = []
    for kind, n, L, P in (("scaling", 40_000, 6, 64), ("offset", 40_000, 6, 64), ("gauss", 400_000, 6, 64),
                          ("feature", 40_000, 1, 256)):
        books, x = scenes.rvq_problem(kind, n, L, P, seed=1)
        b, xx = _up(books, dev), _up(x, dev)
        D = x.shape[1]
        dbooks = torch.zeros_like(b)
        ms = _timed(lambda: vcgs.rvq_assign(b, xx, dbooks=dbooks, grad=True), steps, warmup)
        flops = 2.0 * n * L * P * D
        rows.append({"kind": kind, "n": n, "stages": L, "codes": P, "dim": D, "ms": round(ms, 4),
                     "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
                     "frac_fp32": round(flops / (ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4)})
    return {"workload": "R-VQ of the room map: anchor scaling (3-d) and offsets (30-d), 64 codes x 6 stages, "
                        "40k anchors; per-Gaussian log-scale + rotation (7-d), 64 x 6, 400k Gaussians; "
                        "anchor features (32-d), 256 codes (1-byte), 40k anchors",
            "rows": rows}


def track_section(args, dev, steps=20, warmup=5):
    """One tracking iteration (eq. (21)) and one BA-style step on the room:
    the map is fixed and decoded once; the observed frame is the render at the
    true pose, its depth normalised by alpha where alpha >= 0.5 and 15% missing.  Tracking: render at a perturbed
    pose, silhouette-masked squared colour + depth loss, backward to the pose,
    ICP against the observed depth (every 2nd pixel, tau 5 cm), pose gradient
    summed.  BA step: render, L1 loss + 0.2 SSIM, backward."""
    import numpy as np
    import torch
    from paper_2403_11247_amd import scenes, vcgs
    a = scenes.room_anchors(40000, k=10)
    m = scenes.room_mlp(seed=0)
    A = [_up(x, dev) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    G = vcgs.decode_anchors(*A)
    gs = [G[f] for f in F]
    cam, pose = scenes.room_camera()
    tC, tD, tA, _ = vcgs.render_forward(*gs, cam, pose, keep_state=False)
    # a sensor-like depth: the alpha-normalised render where the surface is solid, 15% missing
    holes = torch.as_tensor(np.random.default_rng(5).uniform(size=(cam.height, cam.width)) < 0.15, device=dev)
    tD = torch.where(holes | (tA < 0.5), torch.zeros_like(tD), tD / tA.clamp_min(0.5))
    cur = scenes.perturb_pose(pose, 3, trans=0.02, rot_deg=1.0)
    stats = {}

    def track_step():
        C, D, Al, st = vcgs.render_forward(*gs, cam, cur)
        loss, dlc, dld = vcgs.track_loss(C, D, Al, tC, tD, lam_d=1.0, norm=2)
        _, dpose = vcgs.render_backward(st, *gs, cam, cur, dlc, dld, None)
        l_icp, _, dpose, matched = vcgs.icp_loss(gs[0], cam, cur, tD, tau=0.05, stride=2, weight=0.1, dpose=dpose)
        st.free()
        stats["matched"] = matched
        return loss, l_icp, dpose

    def ba_step():
        C, D, Al, st = vcgs.render_forward(*gs, cam, cur)
        loss, dlc, dld = vcgs.l1_loss(C, D, tC, tD, 0.5)
        l_s, dlc = vcgs.ssim_loss(C, tC, weight=0.2, dl_dcolor=dlc)
        grads, dpose = vcgs.render_backward(st, *gs, cam, cur, dlc, dld, None)
        st.free()
        return loss, l_s, grads, dpose

    ms_t = _timed(track_step, steps, warmup)
    ms_b = _timed(ba_step, steps, warmup)
    C, D, Al, _ = vcgs.render_forward(*gs, cam, cur, keep_state=False)
    ms_l = _timed(lambda: vcgs.track_loss(C, D, Al, tC, tD), steps, warmup)
    ms_i = _timed(lambda: vcgs.icp_loss(gs[0], cam, cur, tD, tau=0.05, stride=2), steps, warmup)
    ms_s = _timed(lambda: vcgs.ssim_loss(C, tC, 0.2), steps, warmup)
    return {"workload": "room 400k Gaussians, 1200x680: tracking iteration (render, masked colour+depth loss, "
                        "backward, ICP every 2nd pixel) and BA step (render, L1 + 0.2 SSIM, backward)",
            "track_ms": round(ms_t, 4), "ba_ms": round(ms_b, 4), "track_loss_ms": round(ms_l, 4),
            "icp_ms": round(ms_i, 4), "ssim_ms": round(ms_s, 4), "icp_matched": int(stats["matched"][0])}


def serve_section(args, dev):
    """Novel-view requests against a 1M-Gaussian room map (100k anchors at
    2 cm): Poisson arrivals at each rate, sizes uniform over 320x240, 640x480,
    1200x680 and 1920x1080, poses uniform in the room; continuous batching
    against one-at-a-time plain rendering of the same trace."""
    import torch
    from paper_2403_11247_amd import scenes, serve, vcgs
    gd = _decoded_map(100000, 0.02, 4, dev)
    n = int(gd[3].shape[0])
    # pairs-per-pixel estimate from a few plain renders
    cal = scenes.serve_trace(8, qps=100.0, seed=99)
    ppp = 0.0
    for _, c, p in cal:
        _, _, _, st = vcgs.render_forward(*gd, c, p)
        ppp = max(ppp, st.view()["n_pairs"] / (c.width * c.height))
        st.free()
    torch.cuda.synchronize()
    cfg = dict(max_views=16, slots=2, pair_budget=192 << 20, pairs_per_pixel=max(ppp * 1.25, 0.5))
    srv = vcgs.Server(*gd, **cfg)
    warm = scenes.serve_trace(32, qps=1e6, seed=98)
    serve.replay(srv, warm)
    serve.replay_plain(gd, warm[:8])
    rates = []
    for q in [float(x) for x in args.serve_qps.split(",") if x]:
        tr = scenes.serve_trace(args.serve_requests, qps=q, seed=11)
        r_b = serve.replay(srv, tr)
        r_p = serve.replay_plain(gd, tr)
        rates.append({"qps": q, "batched": r_b, "plain": r_p})
        print(f"serve qps {q:g}: batched p50 {r_b['p50_ms']} p99 {r_b['p99_ms']} ms, "
              f"plain p50 {r_p['p50_ms']} p99 {r_p['p99_ms']} ms", file=sys.stderr, flush=True)
    tr = serve.saturate(scenes.serve_trace(args.serve_requests, qps=100.0, seed=12))
    sat_b = serve.replay(srv, tr)
    sat_p = serve.replay_plain(gd, tr)
    srv.close()
    # the same trace with the view-dependent decode: every request decodes the
    # 1M Gaussians at its own camera centre
    a = scenes.room_anchors(100000, k=10, spacing=0.02, seed=4)
    m = scenes.room_mlp_view(seed=4)
    A = [_up(x, dev) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    vsrv = vcgs.Server.from_anchors(*A, **cfg)
    serve.replay(vsrv, warm)
    serve.replay_plain(None, warm[:8], anchors=A)
    vq = 200.0
    trq = scenes.serve_trace(args.serve_requests, qps=vq, seed=11)
    v_rate = {"qps": vq, "batched": serve.replay(vsrv, trq), "plain": serve.replay_plain(None, trq, anchors=A)}
    v_b = serve.replay(vsrv, tr)
    v_p = serve.replay_plain(None, tr, anchors=A)
    vsrv.close()
    return {"workload": "room 100k anchors x 10 at 2 cm (1M Gaussians), Poisson arrivals, sizes uniform over "
                        "320x240/640x480/1200x680/1920x1080, poses uniform in the room, forward only",
            "gaussians": n, "requests_per_rate": args.serve_requests,
            "server": {k: cfg[k] for k in ("max_views", "slots", "pair_budget")},
            "pairs_per_pixel_est": round(cfg["pairs_per_pixel"], 3),
            "rates": rates,
            "saturated": {"batched_mpix_s": sat_b["mpix_s"], "plain_mpix_s": sat_p["mpix_s"],
                          "speedup": round(sat_b["mpix_s"] / max(sat_p["mpix_s"], 1e-9), 2),
                          "views_per_pass": sat_b["views_per_pass"]},
            "view_dependent": {"workload": "the same traces with the view-dependent decode (eqs. (8)-(9)): each "
                                           "request decodes the 1M Gaussians at its own camera centre",
                               "rate": v_rate,
                               "saturated": {"batched_mpix_s": v_b["mpix_s"], "plain_mpix_s": v_p["mpix_s"],
                                             "speedup": round(v_b["mpix_s"] / max(v_p["mpix_s"], 1e-9), 2),
                                             "views_per_pass": v_b["views_per_pass"]}}}


def main():
    args = parse()
    if args.cpu_baseline_child:  # the oracle only; no GPU in this process
        print(json.dumps(cpu_baseline_run(args.cpu_budget_s)), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is design-only",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2403_11247_amd import vcgs
    from paper_2403_11247_amd.vcgs import (decode_anchors, decode_anchors_backward, l1_loss, render_backward,
                                           render_forward)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.only in ("ba", "ba_view", "serve", "view", "mask", "codebook", "rvq", "track"):
        res = {"ba": ba_section, "serve": serve_section, "view": view_decode_section,
               "mask": mask_step_section, "rvq": rvq_section, "track": track_section,
               "ba_view": ba_view_section, "codebook": codebook_section}[args.only](args, dev)
        print(json.dumps({args.only: res}), flush=True)
        return
    if args.only == "main":
        args.no_ba = args.no_serve = args.no_cpu_baseline = True
    a, m, cam, pose, tpose = room_inputs()

    def up(x, dt=torch.float32):
        return torch.as_tensor(np.ascontiguousarray(x)).to(dev, dt)

    A = [up(x) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    F = ("mean", "scale", "quat", "opacity", "color")
    G0 = decode_anchors(*A)
    tC, tD, _, _ = render_forward(*[G0[f] for f in F], cam, tpose, keep_state=False)
    torch.cuda.synchronize()

    def step():
        G = decode_anchors(*A)
        C, D, Al, st = render_forward(*[G[f] for f in F], cam, pose)
        loss, dlc, dld = l1_loss(C, D, tC, tD, 0.5)
        grads, dpose = render_backward(st, *[G[f] for f in F], cam, pose, dlc, dld, None)
        ag = decode_anchors_backward(*A, grads)
        st.free()
        return loss, dpose, ag

    # launch configuration of the compositing kernels for this workload (autotuner)
    from paper_2403_11247_amd import autotune
    tuned, tune_table = autotune.tune_fn(step, f"plain:{cam.width}x{cam.height}:n={G0['opacity'].shape[0]}",
                                         backward=True, reps=3)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # work counts of one step (untimed): visible Gaussians, pairs, compositing evaluations
    vcgs.count_enable(True)
    G = decode_anchors(*A)
    C, D, Al, st = render_forward(*[G[f] for f in F], cam, pose)
    loss, dlc, dld = l1_loss(C, D, tC, tD, 0.5)
    render_backward(st, *[G[f] for f in F], cam, pose, dlc, dld, None)
    torch.cuda.synchronize()
    counts = vcgs.count_read()
    vcgs.count_enable(False)
    view = st.view()
    P = int(view["n_pairs"])
    nvis = int((view["count"] > 0).sum().item())
    n = int(G["opacity"].shape[0])
    st.free()

    # stage times (untimed): every stage's launches bracketed by HIP events
    vcgs.profile_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = vcgs.profile_read()
    vcgs.profile_enable(False)
    per_step = {k: v[0] / max(args.steps, 1) for k, v in prof.items() if v[1] > 0}
    dom = max(per_step, key=per_step.get)

    # timed region: events around the dominant kernel only (two per launch)
    vcgs.profile_stages([dom])
    vcgs.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof_dom = vcgs.profile_read()[dom]
    vcgs.profile_enable(False)
    vcgs.profile_stages(None)

    # per-step latency distribution, after the timed region: HIP events around single steps
    lat_ev = []
    for _ in range(max(args.steps, 50)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        lat_ev.append((e0, e1))
    torch.cuda.synchronize()
    lat = sorted(a_.elapsed_time(b_) for a_, b_ in lat_ev)
    step_latency = {"p50": round(lat[len(lat) // 2], 4), "p99": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 4),
                    "steps": len(lat)}

    ms = (t1 - t0) * 1e3 / args.steps
    mpix = cam.width * cam.height / (ms * 1e-3) / 1e6
    launches = prof_dom[1]
    avg_ms = prof_dom[0] / launches
    na = a.n
    if dom in ("composite", "composite_bwd"):
        units = counts["fwd_evals"] if dom == "composite" else counts["bwd_evals"]
        per_unit = FLOP_EVAL_FWD if dom == "composite" else FLOP_EVAL_BWD
        ach = units * per_unit / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                "flop_per_eval": per_unit, "evals_per_launch": int(units)}
    else:
        b = stage_bytes(dom, n, nvis, P, na, cam.width, cam.height,
                        ((cam.width + 15) // 16) * ((cam.height + 15) // 16))
        ach = b / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    roof["traffic"] = measured_traffic(dom)
    roof["kernel"] = dom
    roof["avg_ms"] = round(avg_ms, 4)
    # HBM roofline fraction of every memory-bound stage (algorithmic bytes / time / peak)
    tiles = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    hbm_stages = {}
    for st_name, ms_step in per_step.items():
        b = stage_bytes(st_name, n, nvis, P, na, cam.width, cam.height, tiles)
        if b and ms_step > 0:
            hbm_stages[st_name] = round(b / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    out = {"metric": "fwd+bwd Mpix/s (300k Gaussians, 1200x680)", "value": round(mpix, 3), "unit": "Mpix/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "room 6x5x3 m, 40k voxel anchors x 10 offsets (400k Gaussians), one 1200x680 view, "
                                  "L1 colour + 0.5 L1 depth, grads to features/MLP/offsets/scalings/pose",
                      "gaussians": n, "visible": nvis, "pairs": P, "pixels": cam.width * cam.height},
           "roofline": roof,
           "autotune": {"best": tuned, "candidates": len(tune_table),
                        "spread_ms": [round(min(t for _, t in tune_table) * 1e3, 3),
                                      round(max(t for _, t in tune_table) * 1e3, 3)] if tune_table else None},
           "step_latency_ms": step_latency,
           "stages_ms": {k: round(v, 4) for k, v in per_step.items()},
           "stages_hbm_frac": hbm_stages,
           "counts": counts}
    if args.copy_probe_mb > 0:
        src = torch.empty(args.copy_probe_mb << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 4
    if args.only != "main":
        out["view_decode_step"] = view_decode_section(args, dev)
        out["mask_step"] = mask_step_section(args, dev)
        out["codebook_step"] = codebook_section(args, dev)
        out["rvq"] = rvq_section(args, dev)
        out["tracking"] = track_section(args, dev)
    if not args.no_ba:
        out["ba_window"] = ba_section(args, dev)
        if args.only != "main":
            out["ba_window_view_decode"] = ba_view_section(args, dev)
    if not args.no_serve:
        out["serving"] = serve_section(args, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget_s)
    if args.stages:
        for k, v in sorted(per_step.items(), key=lambda kv: -kv[1]):
            print(f"{k:16s} {v:8.4f} ms/step", file=sys.stderr)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
