"""ctypes front end of the C oracle (raster.c).  Test infrastructure only.

``render`` follows the method's steps in order: FP32 keys (depth bits, tile
rectangles), pairs sorted by (tile << 32 | depth bits, gid), per-tile ranges,
FP64 projection (eqs. 2-3), FP64 front-to-back compositing (eqs. 16-18).
``render_backward`` is the exact FP64 derivative of the same sums, chained
through the projection to the Gaussian attributes and the camera pose.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


class OCamera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("z_near", ctypes.c_float), ("tile", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = ctypes.CDLL(_build.LIB)
        _lib.orc_pair_count.restype = ctypes.c_int64
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _cam(cam):
    return OCamera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, cam.z_near, cam.tile)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def tiles_of(cam):
    return (cam.width + cam.tile - 1) // cam.tile, (cam.height + cam.tile - 1) // cam.tile


def keys(g, cam, pose):
    """FP32 key path.  Returns depth_bits (u32, 0xFFFFFFFF when culled),
    rect (n, 4) = (tx0, ty0, tx1, ty1) inclusive, and the tile count."""
    n = g.n
    db = np.empty(n, np.uint32)
    rect = np.empty((n, 4), np.int32)
    cnt = np.empty(n, np.int32)
    c = _cam(cam)
    m, s, q, o = (_c(x, np.float32) for x in (g.mean, g.scale, g.quat, g.opacity))
    R, t = _c(pose.R, np.float32), _c(pose.t, np.float32)
    lib().orc_keys(ctypes.c_int64(n), _p(m), _p(s), _p(q), _p(o), ctypes.byref(c), _p(R), _p(t),
                   _p(db), _p(rect), _p(cnt))
    return db, rect, cnt


def sorted_pairs(depth_bits, rect, count, cam):
    """All (key, gid) pairs, sorted by key then gid."""
    n = count.shape[0]
    P = int(lib().orc_pair_count(ctypes.c_int64(n), _p(count)))
    k = np.empty(max(P, 1), np.uint64)
    gid = np.empty(max(P, 1), np.uint32)
    tx, _ = tiles_of(cam)
    lib().orc_sort_pairs(ctypes.c_int64(n), _p(depth_bits), _p(rect), _p(count), ctypes.c_int32(tx),
                         _p(k), _p(gid))
    return k[:P], gid[:P]


def tile_ranges(keys_sorted, cam):
    tx, ty = tiles_of(cam)
    rng = np.empty((tx * ty, 2), np.uint32)
    ks = _c(keys_sorted, np.uint64)
    lib().orc_tile_ranges(ctypes.c_int64(ks.shape[0]), _p(ks), ctypes.c_int32(tx * ty), _p(rng))
    return rng


SPLAT = 12


def project(g, cam, pose):
    """FP64 splat parameters (n, 12): u, v, conic A, B, C, camera depth,
    condition number of Sigma' + 0.3 I, and five zeros (no decision form)."""
    n = g.n
    out = np.empty((n, SPLAT), np.float64)
    m, s, q = (_c(x, np.float64) for x in (g.mean, g.scale, g.quat))
    R, t = _c(pose.R, np.float64), _c(pose.t, np.float64)
    c = _cam(cam)
    lib().orc_project(ctypes.c_int64(n), _p(m), _p(s), _p(q), ctypes.byref(c), _p(R), _p(t), _p(out))
    return out


def decision_form(g, cam, pose, splat):
    """Fills slots 7-11 of ``splat`` in place with the decision form: the
    eigen form of the binary32 footprint covariance of the key path, on which
    the threshold decisions (1/255, 0.99, the stop) are taken."""
    m, s, q, o = (_c(x, np.float32) for x in (g.mean, g.scale, g.quat, g.opacity))
    R, t = _c(pose.R, np.float32), _c(pose.t, np.float32)
    c = _cam(cam)
    assert splat.flags.c_contiguous and splat.dtype == np.float64 and splat.shape == (g.n, SPLAT)
    lib().orc_decision_form(ctypes.c_int64(g.n), _p(m), _p(s), _p(q), _p(o), ctypes.byref(c), _p(R), _p(t),
                            _p(splat))
    return splat


def render(g, cam, pose, bg=(0.0, 0.0, 0.0), decisions="fp32"):
    """Forward render.  Returns a dict with the FP32 keys, the sorted pairs,
    the tile ranges, and FP64 colour (3,H,W), depth, alpha, final
    transmittance, contributor count and ambiguity flags (H, W).
    decisions="fp32" takes the threshold decisions on the binary32 footprint
    covariance (``decision_form``); "fp64" on the FP64 footprint."""
    db, rect, cnt = keys(g, cam, pose)
    ks, gids = sorted_pairs(db, rect, cnt, cam)
    rng = tile_ranges(ks, cam)
    splat = project(g, cam, pose)
    if decisions == "fp32":
        decision_form(g, cam, pose, splat)
    else:
        assert decisions == "fp64", decisions
    W, H = cam.width, cam.height
    C = np.empty((3, H, W)); D = np.empty((H, W)); A = np.empty((H, W)); T = np.empty((H, W))
    nc = np.empty((H, W), np.int32); fl = np.empty((H, W), np.uint8)
    o, col = _c(g.opacity, np.float64), _c(g.color, np.float64)
    bgv = np.asarray(bg, np.float64)
    c = _cam(cam)
    lib().orc_render_fwd(ctypes.c_int64(g.n), _p(splat), _p(o), _p(col), ctypes.byref(c), _p(bgv),
                         _p(rng), _p(gids), _p(C), _p(D), _p(A), _p(T), _p(nc), _p(fl))
    return dict(depth_bits=db, rect=rect, count=cnt, keys=ks, gids=gids, ranges=rng, splat=splat,
                color=C, depth=D, alpha=A, T_final=T, n_contrib=nc, flags=fl, bg=bgv)


def variants(g, cam, fwd, pixels, maxv=64):
    """Every outcome an FP32 renderer may legitimately produce at the given
    flat pixel indices of a forward result ``fwd``: one per combination of the
    pixel's ambiguous threshold decisions (alpha >= 1/255, or the stop at
    T < 1e-4, within FP32 noise) taken either way.  Returns (vals, nvar):
    vals (npx, maxv, 7) = (C0, C1, C2, D, A, T_final, n_contrib) per variant,
    variant 0 the FP64 decisions; nvar (npx,) = number of variants, -1 when a
    pixel has more than maxv."""
    pix = _c(pixels, np.int64)
    npx = pix.shape[0]
    vals = np.full((max(npx, 1), maxv, 7), np.nan)
    nvar = np.zeros(max(npx, 1), np.int32)
    o, col = _c(g.opacity, np.float64), _c(g.color, np.float64)
    c = _cam(cam)
    lib().orc_variants(ctypes.c_int64(g.n), _p(fwd["splat"]), _p(o), _p(col), ctypes.byref(c), _p(fwd["bg"]),
                       _p(fwd["ranges"]), _p(fwd["gids"]), ctypes.c_int64(npx), _p(pix), ctypes.c_int32(maxv),
                       _p(vals), _p(nvar))
    return vals[:npx], nvar[:npx]


def decision_hash(g, cam, fwd, splat=None, opacity=None):
    """Per-pixel hash (H, W) uint64 of which tile-list entries contribute and
    where the pixel stops, over the tile lists of ``fwd``; ``splat`` and
    ``opacity`` replace the footprints of ``fwd`` when given (same lists)."""
    sp = fwd["splat"] if splat is None else _c(splat, np.float64)
    o = _c(g.opacity if opacity is None else opacity, np.float64)
    col = _c(g.color, np.float64)
    out = np.empty((cam.height, cam.width), np.uint64)
    c = _cam(cam)
    lib().orc_decision_hash(ctypes.c_int64(g.n), _p(sp), _p(o), _p(col), ctypes.byref(c), _p(fwd["ranges"]),
                            _p(fwd["gids"]), _p(out))
    return out


def hit_counts(g, cam, fwd):
    """Per-Gaussian hit counts (eq. (13), h) of a forward result ``fwd`` of
    ``render``, and per-Gaussian ambiguity bounds (flagged pixels whose tile
    list holds the Gaussian)."""
    hits = np.empty(g.n, np.uint32)
    amb = np.empty(g.n, np.uint32)
    o = _c(g.opacity, np.float64)
    c = _cam(cam)
    lib().orc_hit_counts(ctypes.c_int64(g.n), _p(fwd["splat"]), _p(o), ctypes.byref(c), _p(fwd["ranges"]),
                         _p(fwd["gids"]), _p(np.ascontiguousarray(fwd["flags"])), _p(hits), _p(amb))
    return hits, amb


def render_backward(g, cam, pose, fwd, dl_dc, dl_dd, dl_da, variant=None):
    """Exact FP64 gradients of sum(dl_dc*C + dl_dd*D + dl_da*A) with respect
    to mean, scale, quat, opacity, colour (same shapes as the inputs) and the
    pose tangent xi = (rho, phi) under left perturbation.  ``variant`` (H, W)
    int32, optional: per pixel, which of its ``variants`` the derivative
    follows (0 = every decision as in FP64)."""
    n = g.n
    g2 = np.empty((n, 10))
    o, col = _c(g.opacity, np.float64), _c(g.color, np.float64)
    dc, dd, da = _c(dl_dc, np.float64), _c(dl_dd, np.float64), _c(dl_da, np.float64)
    c = _cam(cam)
    var = None if variant is None else _c(variant, np.int32)
    lib().orc_render_bwd_2d(ctypes.c_int64(n), _p(fwd["splat"]), _p(o), _p(col), ctypes.byref(c),
                            _p(fwd["bg"]), _p(fwd["ranges"]), _p(fwd["gids"]), _p(dc), _p(dd), _p(da),
                            None if var is None else _p(var), _p(g2))
    vis = (fwd["count"] > 0).astype(np.int32)
    m, s, q = (_c(x, np.float64) for x in (g.mean, g.scale, g.quat))
    R, t = _c(pose.R, np.float64), _c(pose.t, np.float64)
    dm = np.empty((3, n)); ds = np.empty((3, n)); dq = np.empty((4, n)); do = np.empty(n); dcol = np.empty((3, n))
    dpose = np.empty(6)
    lib().orc_project_bwd(ctypes.c_int64(n), _p(m), _p(s), _p(q), ctypes.byref(c), _p(R), _p(t), _p(vis),
                          _p(g2), _p(dm), _p(ds), _p(dq), _p(do), _p(dcol), _p(dpose))
    return dict(mean=dm, scale=ds, quat=dq, opacity=do, color=dcol, pose=dpose, g2=g2)
