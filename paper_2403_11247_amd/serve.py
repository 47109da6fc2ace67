"""Open-loop replay of a request trace against the continuous-batching server
and against a one-at-a-time plain renderer.

A trace is a list of (arrival seconds, camera, pose) in arrival order.  Time
zero is the start of the replay; a request's latency runs from its scheduled
arrival to the moment the host sees its images complete, so any delay in
submitting it is counted too.
"""
from __future__ import annotations

import gc
import time

import numpy as np
import torch

from . import vcgs


def _stats(lat, pixels, t_first, t_last):
    lat = np.asarray(lat)
    span = max(t_last - t_first, 1e-9)
    return {"requests": int(lat.size),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "mean_ms": round(float(lat.mean()) * 1e3, 3),
            "max_ms": round(float(lat.max()) * 1e3, 3),
            "mpix_s": round(pixels / span / 1e6, 2),
            "span_s": round(span, 3)}


def replay(server: "vcgs.Server", trace, poll_us=200, ring=64):
    """Submits each request at its arrival time and polls the server until all
    complete.  Returns latency percentiles, throughput and server counters.
    Output images come from a ring of `ring` buffer sets per image size,
    allocated before the replay starts, as a serving loop reuses its image
    buffers (more sets than the server can have in running passes, so no two
    running requests share one); an arrival costs only the submission and the
    launch."""
    n = len(trace)
    lat = [0.0] * n
    pending = {}
    st0 = server.stats()
    pixels = sum(int(c.width) * int(c.height) for _, c, _ in trace)
    dev = server.dev
    pools, seen, outs = {}, {}, []
    for _, c, _ in trace:
        key = (int(c.height), int(c.width))
        k = seen.get(key, 0)
        seen[key] = k + 1
        pool = pools.setdefault(key, [])
        if k < ring:
            pool.append((torch.empty((3,) + key, device=dev), torch.empty(key, device=dev), torch.empty(key, device=dev)))
        outs.append(pool[k % ring])
    torch.cuda.synchronize()
    # no collector pauses inside the timed loop (a full collection of a large
    # process stalls the host for tens of milliseconds)
    gc.collect()
    gc.disable()
    try:
        t0 = time.perf_counter()
        t_last = _replay_loop(server, trace, outs, pending, lat, poll_us, t0)
    finally:
        gc.enable()
    out = _stats(lat, pixels, trace[0][0], t_last)
    st1 = server.stats()
    out.update({k: st1[k] - st0[k] for k in ("passes", "reruns")})
    out["views_per_pass"] = round(n / max(out["passes"], 1), 2)
    return out


def _replay_loop(server, trace, outs, pending, lat, poll_us, t0):
    n = len(trace)
    i = 0
    t_last = 0.0
    while i < n or pending:
        now = time.perf_counter() - t0
        if not pending and i < n and trace[i][0] > now:
            # nothing in flight: wait for the next arrival as the plain loop does
            while time.perf_counter() - t0 < trace[i][0]:
                pass
            now = time.perf_counter() - t0
        while i < n and trace[i][0] <= now:
            _, cam, pose = trace[i]
            tk, out = server.submit(cam, pose, out=outs[i])
            pending[tk] = (i, out)
            i += 1
        wait_us = poll_us if i >= n else max(0.0, min(poll_us * 1e-6, trace[i][0] - now)) * 1e6
        done = server.progress(timeout_us=int(wait_us))
        if done:
            t_done = time.perf_counter() - t0
            for tk in done:
                j, _ = pending.pop(tk)
                lat[j] = t_done - trace[j][0]
            t_last = t_done
    return t_last


def replay_plain(gauss, trace, anchors=None):
    """FIFO baseline: one request at a time with the plain forward render
    (which sizes its pair buffers with one synchronisation) and a wait for its
    completion before the next starts.  With anchors (the decode inputs, W1
    (32, 36)) each request first decodes the map at its own camera centre and
    gauss is ignored."""
    n = len(trace)
    lat = [0.0] * n
    pixels = sum(int(c.width) * int(c.height) for _, c, _ in trace)
    gc.collect()
    gc.disable()
    try:
        t_last = _plain_loop(gauss, trace, anchors, lat)
    finally:
        gc.enable()
    return _stats(lat, pixels, trace[0][0], t_last)


def _plain_loop(gauss, trace, anchors, lat):
    t0 = time.perf_counter()
    t_last = 0.0
    for j, (arr, cam, pose) in enumerate(trace):
        while time.perf_counter() - t0 < arr:
            pass
        if anchors is not None:
            G = vcgs.decode_anchors(*anchors, cam_centre=vcgs.camera_centre(pose))
            gauss = [G[f] for f in ("mean", "scale", "quat", "opacity", "color")]
        vcgs.render_forward(*gauss, cam, pose, keep_state=False)
        torch.cuda.synchronize()
        t_last = time.perf_counter() - t0
        lat[j] = t_last - arr
    return t_last


def saturate(trace):
    """The same requests all arriving at time zero (closed system): the
    throughput ceiling of either server."""
    return [(0.0, c, p) for _, c, p in trace]
