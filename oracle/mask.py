"""Mask training step oracle (numpy float64).  Test infrastructure only.

Sec. 3.3 of the paper, eq. (13): the mask loss L_m is the mean of
sigmoid(m_n) over the Gaussians of the window; with the frustum restriction
only the Gaussians in the current view's frustum (a non-empty tile rectangle)
are in the window and get a gradient.  Gaussians are removed at the end of a
window when their mask is off (sigmoid(m) <= eps, eq. (11)) or their hit count
h is below a minimum (the paper evaluates "hit frequency in conjunction with
the learned mask" without a number; the minimum is a parameter).
"""
from __future__ import annotations

import numpy as np


def _sig(x):
    return 1.0 / (1.0 + np.exp(-x))


def mask_loss(mask_logit, in_frustum, weight=1.0):
    """(L_m, dL_m/dm) with L_m = weight * mean over the frustum of sigmoid(m)."""
    m = np.asarray(mask_logit, np.float64)
    inf = np.asarray(in_frustum, bool)
    cnt = int(inf.sum())
    if cnt == 0:
        return 0.0, np.zeros_like(m)
    s = _sig(m)
    loss = weight * s[inf].sum() / cnt
    grad = np.where(inf, weight * s * (1 - s) / cnt, 0.0)
    return loss, grad


def prune(mask_logit, hits, eps=0.01, min_hits=1):
    """Kept flags and the kept indices in order (a stable compaction)."""
    keep = (_sig(np.asarray(mask_logit, np.float64)) > eps) & (np.asarray(hits) >= min_hits)
    return keep, np.nonzero(keep)[0].astype(np.uint32)
