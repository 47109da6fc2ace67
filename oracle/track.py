"""Tracking and bundle-adjustment losses (numpy float64).  Test infrastructure only.

Sec. 3.5 of the paper:
  eq. (19)  colour loss over all N pixels and depth loss over the rays R with a
            depth observation (squared errors, or absolute errors as in the
            workload's L1 form);
  eq. (20)  ICP loss sum_i w_i |R p_i + t - q_i|^2, p_i a Gaussian centre and
            q_i its closest observed point;
  eq. (21)  tracking loss: the per-pixel terms only where the rendered
            silhouette S(p) = sum_i f_i prod_{j<i}(1 - f_j) exceeds 0.99, plus
            the ICP term;
  BA        the same plus an SSIM term on the colour render.

Readings (the paper is silent or garbled here; listed in the design notes):
  - eq. (21) puts the indicator inside the pixel sum; L_icp has no pixel, so
    L_t = sum_p 1[S>0.99] (l_c(p) + lam_d l_d(p)) + lam_icp L_icp, with
    l_c(p) = |C^(p) - C(p)|^2 / N (summed over channels) and
    l_d(p) = (D^(p) - D(p))^2 / |R| for p in R (D > 0 observed), N = H W;
  - q_i: nearest point of the observed depth map back-projected at pixel
    centres, taking every s-th pixel in each direction (s = 1: all); w_i = 1 if
    that distance is below tau, else 0; camera frame p_c = R p + t;
  - pose gradient under the left perturbation p_c <- p_c + rho + phi x p_c:
    dL/drho = sum g_i, dL/dphi = sum p_c,i x g_i, g_i = 2 w_i (p_c,i - q_i);
    q_i is held fixed (no gradient through the association);
  - SSIM: Wang et al. (2004) with an 11 x 11 Gaussian window, sigma 1.5,
    C1 = 0.01^2, C2 = 0.03^2, per channel, zero padding outside the image,
    L_ssim = 1 - mean over channels and pixels.
"""
from __future__ import annotations

import numpy as np

SIL_THRESH = 0.99


def track_loss(C, D, A, tC, tD, lam_d=1.0, norm=2, thresh=SIL_THRESH):
    """Masked colour + depth loss of eqs. (19), (21).  C, tC (3, H, W); D, tD,
    A (H, W).  Returns (loss, dL/dC, dL/dD); norm 2 = squared, 1 = absolute
    (subgradient sign(0) = 0)."""
    C, D, A = (np.asarray(a, np.float64) for a in (C, D, A))
    tC, tD = np.asarray(tC, np.float64), np.asarray(tD, np.float64)
    H, W = D.shape
    N = H * W
    m = (A > thresh).astype(np.float64)
    valid = tD > 0
    nR = int(valid.sum())
    ec = C - tC
    ed = np.where(valid, D - tD, 0.0)
    if norm == 2:
        lc = (m[None] * ec ** 2).sum() / N
        gc = m[None] * 2.0 * ec / N
        ld = (m * ed ** 2).sum() / nR if nR else 0.0
        gd = m * 2.0 * ed / nR if nR else np.zeros_like(D)
    else:
        lc = (m[None] * np.abs(ec)).sum() / N
        gc = m[None] * np.sign(ec) / N
        ld = (m * np.abs(ed)).sum() / nR if nR else 0.0
        gd = m * np.sign(ed) / nR if nR else np.zeros_like(D)
    return lc + lam_d * ld, gc, lam_d * gd


def backproject(depth, cam, stride=1):
    """Observed points (camera frame) at pixel centres with depth > 0, every
    ``stride``-th pixel in each direction.  Returns (M, 3)."""
    depth = np.asarray(depth, np.float64)
    H, W = depth.shape
    v, u = np.mgrid[0:H:stride, 0:W:stride]
    z = depth[v, u]
    ok = z > 0
    u, v, z = u[ok], v[ok], z[ok]
    x = (u + 0.5 - cam.cx) / cam.fx * z
    y = (v + 0.5 - cam.cy) / cam.fy * z
    return np.stack([x, y, z], 1)


def icp(means, pose, depth, cam, tau, stride=1, chunk=2048):
    """ICP term of eq. (20) by brute-force nearest neighbours.  means (3, n)
    world; pose (R, t).  Returns dict(loss, dmeans (3, n), dpose (6,) =
    (rho, phi), w (n,), dist (n,) nearest distance, nn (n,) index into the
    back-projected points (-1 if none), pts (M, 3), second (n,) second-nearest
    distance)."""
    R = np.asarray(pose.R, np.float64).reshape(3, 3)
    t = np.asarray(pose.t, np.float64)
    mu = np.asarray(means, np.float64)
    n = mu.shape[1]
    pc = (R @ mu).T + t
    Q = backproject(depth, cam, stride)
    dist = np.full(n, np.inf)
    second = np.full(n, np.inf)
    nn = np.full(n, -1, np.int64)
    if len(Q):
        for s in range(0, n, chunk):
            d2 = ((pc[s:s + chunk, None, :] - Q[None, :, :]) ** 2).sum(-1)
            k = d2.argmin(1)
            nn[s:s + chunk] = k
            dist[s:s + chunk] = np.sqrt(d2[np.arange(len(k)), k])
            if d2.shape[1] > 1:
                second[s:s + chunk] = np.sqrt(np.partition(d2, 1, axis=1)[:, 1])
    w = (dist < tau).astype(np.float64)
    q = np.where(nn[:, None] >= 0, Q[np.maximum(nn, 0)], 0.0)
    e = np.where(w[:, None] > 0, pc - q, 0.0)
    loss = float((w * (e ** 2).sum(1)).sum())
    g = 2.0 * e
    dmeans = (g @ R).T
    dpose = np.concatenate([g.sum(0), np.cross(pc, g).sum(0)])
    return dict(loss=loss, dmeans=dmeans, dpose=dpose, w=w, dist=dist, nn=nn, pts=Q, second=second)


def gauss_window(size=11, sigma=1.5):
    x = np.arange(size) - size // 2
    g = np.exp(-x ** 2 / (2.0 * sigma ** 2))
    return g / g.sum()


def _filt(img, g):
    """Zero-padded 'same' correlation with the separable window g x g, as
    explicit shifted sums (rows, then columns)."""
    H, W = img.shape
    r = len(g) // 2
    p = np.zeros((H, W + 2 * r))
    p[:, r:r + W] = img
    tmp = sum(g[k] * p[:, k:k + W] for k in range(len(g)))
    p = np.zeros((H + 2 * r, W))
    p[r:r + H] = tmp
    return sum(g[k] * p[k:k + H] for k in range(len(g)))


C1 = 0.01 ** 2
C2 = 0.03 ** 2


def ssim(x, y, window=11, sigma=1.5):
    """Mean SSIM of images x, y (3, H, W) and the gradient of
    L_ssim = 1 - mean SSIM with respect to x.  Returns (L_ssim, dL/dx, map)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    g = gauss_window(window, sigma)
    Ch, H, W = x.shape
    total = 0.0
    grad = np.zeros_like(x)
    maps = np.zeros_like(x)
    M = Ch * H * W
    for c in range(Ch):
        a, b = x[c], y[c]
        mx, my = _filt(a, g), _filt(b, g)
        sxx = _filt(a * a, g) - mx * mx
        syy = _filt(b * b, g) - my * my
        sxy = _filt(a * b, g) - mx * my
        n1 = 2 * mx * my + C1
        n2 = 2 * sxy + C2
        d1 = mx * mx + my * my + C1
        d2 = sxx + syy + C2
        s = n1 * n2 / (d1 * d2)
        maps[c] = s
        total += s.sum()
        # partial derivatives of s with respect to mx, sxx, sxy at each pixel
        ds_dmx = (2 * my * n2) / (d1 * d2) - s * (2 * mx) / d1
        ds_dsxx = -s / d2
        ds_dsxy = 2 * n1 / (d1 * d2)
        # x enters through mx = G*a, sxx = G*a^2 - mx^2, sxy = G*(a b) - mx my
        A_ = ds_dmx - 2 * mx * ds_dsxx - my * ds_dsxy
        grad[c] = _filt(A_, g) + 2 * a * _filt(ds_dsxx, g) + b * _filt(ds_dsxy, g)
    return 1.0 - total / M, -grad / M, maps
