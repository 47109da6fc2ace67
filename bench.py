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

# Algorithmic work per unit (see the design notes for the derivation).
FLOP_FOOTPRINT = 16     # one (pixel, Gaussian) footprint evaluation incl. the exponential
FLOP_BLEND_FWD = 13     # transmittance update and colour/depth/alpha accumulation
FLOP_BLEND_BWD = 47     # one contributing (pixel, Gaussian) in the adjoint


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--stages", action="store_true", help="also print a per-stage table to stderr")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    return ap.parse_args()


def room_inputs():
    from paper_2403_11247_amd import scenes
    a = scenes.room_anchors(40000, k=10)
    m = scenes.room_mlp()
    cam, pose = scenes.room_camera()
    tpose = scenes.perturb_pose(pose, 2)
    return a, m, cam, pose, tpose


def stage_bytes(stage, n, nvis, P, na, W, H):
    """Algorithmic HBM bytes of one launch of a stage."""
    if stage == "decode":
        return na * (12 + 128 + 12 + 120) + n * 56
    if stage == "preprocess":
        return n * (56 + 16) + nvis * 48
    if stage == "depth_sort":
        return n * 8 + 4 * n * 20
    if stage == "tile_sort":
        return 2 * P * 20 + P * 8
    if stage == "emit":
        return nvis * 20 + P * 8
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


def cpu_baseline(budget_s):
    """The oracle, as it stands, on the same workload: full fwd+bwd steps until
    the time budget is used (at least one)."""
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
            "kind": "oracle",
            "sample": f"{steps} full fwd+bwd step(s) of the room workload (1200x680, 400k Gaussians), "
                      f"{dt:.2f} s each; projection/compositing forward on {threads} OpenMP threads, "
                      f"adjoint single-threaded"}


def main():
    args = parse()
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

    vcgs.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = vcgs.profile_read()
    vcgs.profile_enable(False)

    ms = (t1 - t0) * 1e3 / args.steps
    mpix = cam.width * cam.height / (ms * 1e-3) / 1e6
    per_step = {k: v[0] / max(args.steps, 1) for k, v in prof.items() if v[1] > 0}
    dom = max(per_step, key=per_step.get)
    launches = prof[dom][1]
    avg_ms = prof[dom][0] / launches
    na = a.n
    if dom in ("composite", "composite_bwd"):
        if dom == "composite":
            flop = counts["fwd_evals"] * FLOP_FOOTPRINT + counts["fwd_blends"] * FLOP_BLEND_FWD
        else:
            flop = counts["bwd_evals"] * FLOP_FOOTPRINT + counts["bwd_blends"] * FLOP_BLEND_BWD
        ach = flop / (avg_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None}
    else:
        b = stage_bytes(dom, n, nvis, P, na, cam.width, cam.height)
        ach = b / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    roof["traffic"] = measured_traffic(dom)
    roof["kernel"] = dom
    roof["avg_ms"] = round(avg_ms, 4)

    out = {"metric": "fwd+bwd Mpix/s (300k Gaussians, 1200x680)", "value": round(mpix, 3), "unit": "Mpix/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "room 6x5x3 m, 40k voxel anchors x 10 offsets (400k Gaussians), one 1200x680 view, "
                                  "L1 colour + 0.5 L1 depth, grads to features/MLP/offsets/scalings/pose",
                      "gaussians": n, "visible": nvis, "pairs": P, "pixels": cam.width * cam.height},
           "roofline": roof,
           "stages_ms": {k: round(v, 4) for k, v in per_step.items()},
           "counts": counts}
    if args.copy_probe_mb > 0:
        src = torch.empty(args.copy_probe_mb << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 4
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget_s)
    if args.stages:
        for k, v in sorted(per_step.items(), key=lambda kv: -kv[1]):
            print(f"{k:16s} {v:8.4f} ms/step", file=sys.stderr)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
