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


def compare_images(C, D, A, ref, tol=IMG_TOL, depth_tol=None, g=None, cam=None, pix_state=None):
    """Max errors on unflagged pixels and the flagged count.

    With the Gaussians ``g`` and camera ``cam``, every flagged pixel (a
    threshold decision within FP32 noise) is checked as well: the GPU's
    colour, depth and alpha must equal, within tol, one of the outcomes the
    oracle enumerates for that pixel (each ambiguous decision taken either
    way).  ``pix_state`` = the GPU's (T_final, n_contrib) images narrows the
    match to the outcome with the same contributor count and final
    transmittance; the result's ``variant`` map (H, W) then holds the index of
    the single matching outcome per pixel (0 on unflagged pixels, -1 where
    more than one matches), for the backward to follow."""
    depth_tol = tol if depth_tol is None else depth_tol
    ok = (ref["flags"] & 3) == 0
    C = C.cpu().numpy().astype(np.float64)
    D = D.cpu().numpy().astype(np.float64)
    A = A.cpu().numpy().astype(np.float64)
    ec = np.abs(C - ref["color"])[:, ok].max(initial=0.0)
    ed = np.abs(D - ref["depth"])[ok].max(initial=0.0)
    ea = np.abs(A - ref["alpha"])[ok].max(initial=0.0)
    flagged = int((~ok).sum())
    eflag_c = np.abs(C - ref["color"])[:, ~ok].max(initial=0.0)
    out = dict(color=ec, depth=ed, alpha=ea, flagged=flagged, flagged_color=eflag_c,
               pass_=(ec <= tol and ed <= depth_tol and ea <= tol))
    if g is None or flagged == 0:
        out["variant"] = np.zeros(ok.shape, np.int32)
        out["flagged_unmatched"] = 0
        out["flagged_ambiguous"] = 0
        return out
    from oracle import raster
    pix = np.flatnonzero(~ok.ravel())
    vals, nvar = raster.variants(g, cam, ref, pix)
    assert (nvar > 0).all(), "a flagged pixel has more outcomes than enumerated"
    got = np.stack([C.reshape(3, -1)[0, pix], C.reshape(3, -1)[1, pix], C.reshape(3, -1)[2, pix],
                    D.ravel()[pix], A.ravel()[pix]], axis=1)
    err = np.abs(vals[:, :, :5] - got[:, None, :])
    lim = np.array([tol, tol, tol, depth_tol, tol])
    match = np.all(err <= lim, axis=2) & (np.arange(vals.shape[1])[None, :] < nvar[:, None])
    if pix_state is not None:
        T, nc = (x.cpu().numpy() for x in pix_state)
        Tg, ng = T.ravel()[pix].astype(np.float64), nc.ravel()[pix]
        match &= np.abs(vals[:, :, 5] / np.maximum(Tg[:, None], 1e-30) - 1.0) <= 1e-3
        match &= vals[:, :, 6] == ng[:, None]
    nmatch = match.sum(axis=1)
    variant = np.zeros(ok.shape, np.int32)
    vflat = variant.ravel()
    vflat[pix] = np.where(nmatch == 1, np.argmax(match, axis=1), -1)
    out["variant"] = variant
    out["flagged_unmatched"] = int((nmatch == 0).sum())
    out["flagged_ambiguous"] = int((nmatch > 1).sum())
    out["pass_"] = out["pass_"] and out["flagged_unmatched"] == 0
    return out


def zero_at(up, mask):
    """Copies of the upstream gradients (dC (3,H,W), dD, dA) with zeros where mask."""
    up = [np.array(u, copy=True) for u in up]
    up[0][:, mask] = 0.0
    up[1][mask] = 0.0
    up[2][mask] = 0.0
    return up


def grad_check(name, got, ref, tol=GRAD_REL_TOL, floor=1e-6):
    """The gradient bars: per-tensor relative L2 error <= tol, and element by
    element |got - ref| <= tol |ref| + floor max|ref|.  Returns the L2 error."""
    a = np.asarray(got, np.float64)
    b = np.asarray(ref, np.float64)
    rel = rel_err(a, b)
    bound = tol * np.abs(b) + floor * np.abs(b).max(initial=0.0)
    bad = np.abs(a - b) > bound
    nbad = int(bad.sum())
    if nbad:
        i = np.argmax(np.abs(a - b) - bound)
        say(f"{name}: {nbad} of {b.size} elements outside the element bound; worst got {a.ravel()[i]:.6e} "
            f"ref {b.ravel()[i]:.6e}")
    assert rel <= tol, (name, rel)
    assert nbad == 0, (name, nbad)
    return rel
