"""Autotuner of the compositing launch configuration for a batched window.

The tunable settings are the library's kernel options (vcgs_set_option):
pixels per lane of the forward and backward compositing (1, 2, 4: a 16x16 tile
walked by 4, 2 or 1 waves, i.e. the block's tile shape), per-wave culling of
tile-list entries, the block schedule (linear or XCD-aware), and, at one pixel
per lane, whether a tile's waves merge their gradient sums before the atomics.
None changes a result beyond the order of floating-point sums.  ``tune`` times every candidate on the window as given (eager
passes, median of ``reps``) and leaves the fastest set; a graph captured
afterwards keeps it.  Results are cached per window signature (image sizes,
map size, backward or not).
"""
from __future__ import annotations

import itertools
import json
import os
import time

import torch

from . import vcgs

KEYS = ("ppl_fwd", "ppl_bwd", "cull", "sched", "bwd_merge")
SPACE = {"ppl_fwd": (1, 2, 4), "ppl_bwd": (1, 2, 4), "cull": (1, 0), "sched": (1, 0), "bwd_merge": (0, 1)}

_cache: dict = {}


def signature(win) -> str:
    sizes = ",".join(f"{int(c.width)}x{int(c.height)}" for c in win.cameras)
    return f"n={win.n};views={sizes};bwd={int(win.backward)}"


def current() -> dict:
    return {k: vcgs.get_option(k) for k in KEYS}


def apply(cfg: dict):
    for k in KEYS:
        if k in cfg:
            vcgs.set_option(k, int(cfg[k]))


def candidates(backward=True):
    keys = KEYS if backward else ("ppl_fwd", "cull", "sched")
    for vals in itertools.product(*[SPACE[k] for k in keys]):
        cfg = dict(zip(keys, vals))
        if cfg.get("bwd_merge") and cfg["ppl_bwd"] != 1:
            continue  # merging applies to the one-pixel-per-lane backward only
        yield cfg


def _time(fn, reps):
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    return ts[len(ts) // 2]


def tune_fn(fn, sig, backward=True, reps=3, warmup=1, verbose=False):
    """Pick the fastest option set for an arbitrary pass ``fn`` (e.g. one plain
    forward + backward step); ``sig`` names it in the cache."""
    if sig in _cache:
        apply(_cache[sig])
        return _cache[sig], []
    saved = current()
    table = []
    try:
        for cfg in candidates(backward):
            apply(cfg)
            for _ in range(warmup):
                fn()
            t = _time(fn, reps)
            table.append((dict(cfg), t))
            if verbose:
                print(f"  {cfg} {t * 1e3:.3f} ms", flush=True)
    finally:
        apply(saved)
    best = min(table, key=lambda kv: kv[1])[0]
    apply(best)
    _cache[sig] = best
    return best, table


def tune(win, run_args, reps=3, warmup=1, verbose=False):
    """Pick the fastest option set for ``win`` (a vcgs.BatchWindow, normally
    eager) running ``win.run(*run_args)``.  Returns (best config, table of
    (config, seconds)); the table is empty when the signature was cached."""
    return tune_fn(lambda: win.run(*run_args), signature(win), win.backward, reps, warmup, verbose)


def save(path):
    with open(path, "w") as f:
        json.dump(_cache, f, indent=1, sort_keys=True)


def load(path):
    if os.path.exists(path):
        with open(path) as f:
            _cache.update(json.load(f))
