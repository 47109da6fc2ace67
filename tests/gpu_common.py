"""Helpers shared by the GPU parity tests: device upload, running the HIP path
through the C ABI binding, and comparing against the oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

from paper_2403_11247_amd import scenes

FIELDS = ("mean", "scale", "quat", "opacity", "color")

# Parity bars.  Images: absolute, on pixels whose threshold decisions are not
# within FP32 noise (the oracle flags those).  Gradients: per-tensor relative
# L2 error.
IMG_TOL = 1e-4
GRAD_REL_TOL = 1e-3


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def gauss_dev(g: scenes.Gaussians):
    return [dev(getattr(g, f)) for f in FIELDS]


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def keys_from_state(view, n):
    """(depth bits u32, rect (n,4) int, count) from a GPU state view."""
    db = view["depth_bits"].cpu().numpy().view(np.uint32)
    rect = view["rect"].cpu().numpy().astype(np.int64).reshape(n, 4) & 0xFFFF
    cnt = view["count"].cpu().numpy().view(np.uint32)
    return db, rect, cnt


def compare_keys(view, ref, n, cam):
    """Bit-exact check of depth bits, tile rectangles, counts, the sorted
    Gaussian order and the tile ranges against the oracle."""
    db, rect, cnt = keys_from_state(view, n)
    vis = ref["count"] > 0
    assert np.array_equal(cnt, ref["count"].astype(np.uint32)), "tile counts differ"
    assert np.array_equal(db[vis], ref["depth_bits"][vis]), "depth bits differ"
    assert np.array_equal(rect[vis], ref["rect"][vis].astype(np.int64)), "tile rectangles differ"
    gids = view["gids"].cpu().numpy().view(np.uint32)
    assert gids.shape[0] == ref["gids"].shape[0], "pair count differs"
    assert np.array_equal(gids, ref["gids"]), "sorted Gaussian order differs"
    rng = view["ranges"].cpu().numpy().view(np.uint32)
    assert np.array_equal(rng, ref["ranges"]), "tile ranges differ"
    # the GPU's implied 64-bit keys equal the oracle's sorted keys
    tiles = np.repeat(np.arange(rng.shape[0], dtype=np.uint64), (rng[:, 1] - rng[:, 0]).astype(np.int64))
    keys = (tiles << np.uint64(32)) | db[gids].astype(np.uint64)
    assert np.array_equal(keys, ref["keys"]), "keys differ"


def compare_images(C, D, A, ref, tol=IMG_TOL, depth_tol=None):
    """Returns a dict of max errors on unflagged pixels and the flagged count."""
    depth_tol = tol if depth_tol is None else depth_tol
    ok = (ref["flags"] & 3) == 0
    C = C.cpu().numpy().astype(np.float64)
    D = D.cpu().numpy().astype(np.float64)
    A = A.cpu().numpy().astype(np.float64)
    ec = np.abs(C - ref["color"])[:, ok].max(initial=0.0)
    ed = np.abs(D - ref["depth"])[ok].max(initial=0.0)
    ea = np.abs(A - ref["alpha"])[ok].max(initial=0.0)
    flagged = int((~ok).sum())
    # flagged pixels: both outcomes of a threshold decision are valid; the
    # difference is bounded by one excluded/included footprint
    eflag_c = np.abs(C - ref["color"])[:, ~ok].max(initial=0.0)
    return dict(color=ec, depth=ed, alpha=ea, flagged=flagged, flagged_color=eflag_c,
                pass_=(ec <= tol and ed <= depth_tol and ea <= tol))
