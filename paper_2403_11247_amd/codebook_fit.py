"""Input preparation for the compacted room workload (mask + residual
codebooks, Sec. 3.3-3.4): two-stage residual k-means codebooks of 4096 x 7
entries fit to a decoded map's per-Gaussian (log-scale, quaternion).

This builds the workload's inputs; it is not a step of the rendering path.
It runs Lloyd iterations with plain PyTorch tensor operations on the device
(distances by chunked matrix products, centroids by scatter sums); the
decode that consumes the codebooks is the library's.
"""
from __future__ import annotations

import torch


def _nearest(x, C, chunk=1 << 16):
    """Index of the nearest row of C for every row of x (squared Euclidean)."""
    cc = (C * C).sum(1)
    out = torch.empty(x.shape[0], dtype=torch.int64, device=x.device)
    for i in range(0, x.shape[0], chunk):
        xs = x[i:i + chunk]
        d = cc[None, :] - 2.0 * (xs @ C.t())
        out[i:i + chunk] = d.argmin(1)
    return out


def residual_kmeans(x, stages=2, size=4096, iters=10, seed=0):
    """Residual k-means of x (n, D) float32 on the device: stage l fits `size`
    centroids to the residual left by stages < l (initialised from randomly
    drawn rows, `iters` Lloyd iterations; an empty cluster keeps its centroid).
    Returns (books (stages, size, D) float32, idx (stages, n) int32)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    n, D = x.shape
    books = torch.empty((stages, size, D), device=x.device)
    idx = torch.empty((stages, n), dtype=torch.int32, device=x.device)
    r = x.clone()
    for s in range(stages):
        C = r[torch.randint(0, n, (size,), generator=g).to(x.device)].clone()
        for _ in range(iters):
            a = _nearest(r, C)
            sums = torch.zeros_like(C).index_add_(0, a, r)
            cnt = torch.bincount(a, minlength=size).to(r.dtype)
            C = torch.where(cnt[:, None] > 0, sums / cnt.clamp_min(1.0)[:, None], C)
        a = _nearest(r, C)
        books[s] = C
        idx[s] = a.to(torch.int32)
        r = r - C[a]
    return books, idx


def shape_vectors(G):
    """Per-Gaussian (log-scale, quaternion) rows (n, 7) of a decoded map, the
    vectors the decode's codebooks reproduce."""
    return torch.cat([torch.log(G["scale"]), G["quat"]], 0).t().contiguous()


def psnr(a, b, peak=1.0):
    """Peak signal-to-noise ratio (dB) of image a against b."""
    mse = float(((a - b) ** 2).mean())
    return float("inf") if mse == 0.0 else 10.0 * torch.log10(torch.tensor(peak * peak / mse)).item()
