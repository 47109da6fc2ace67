"""Anchor decode oracle (numpy float64).  Test infrastructure only.

Follows Sec. 3.2 of the paper:
  eq. (7)  mu_i = x_a + O_i . l   (the product read element-wise)
  eq. (8)  {f_a, delta, d} -> {alpha_i, q_i, s_i, c_i}, i = 0..k-1, through an
           MLP: one 2-layer MLP -> 32 ReLU -> k*11.  Without a camera the input
           is the 32-d feature alone (view-independent form); with the camera
           centre x_c it is the 36-d [f_a, delta, d] of eq. (9):
           delta = |x_a - x_c|, d = (x_a - x_c) / delta.
Sec. 3.3 eqs. (11)-(12): binary mask M = 1[sigmoid(m) > eps] in value, with
           the straight-through gradient of sigmoid(m); s_hat = M s,
           alpha_hat = M alpha.
Sec. 3.4 eq. (14), first line: the residual codebook value is the sum of the
           selected code of every stage; here it supplies 3 log-scales and the
           4 quaternion components of each Gaussian.

Activations (the paper names none): sigmoid for opacity and colour, exp for
the log-scales, the quaternion is passed on raw (the renderer normalises it).
Per-offset output layout: [opacity, r, g, b, log s0, log s1, log s2, qw, qx, qy, qz].
"""
from __future__ import annotations

import numpy as np

OUT = 11


def _sig(x):
    return 1.0 / (1.0 + np.exp(-x))


def view_inputs(anchors, cam):
    """Eq. (9): per-anchor viewing distance and unit direction from the camera
    centre, as (na, 4) = [delta, d_x, d_y, d_z]."""
    xa = np.asarray(anchors.xa, np.float64).T
    v = xa - np.asarray(cam, np.float64)[None, :]
    delta = np.sqrt((v * v).sum(1))
    return np.concatenate([delta[:, None], v / delta[:, None]], axis=1)


def mlp_input(anchors, cam=None):
    f = np.asarray(anchors.feat, np.float64)
    return f if cam is None else np.concatenate([f, view_inputs(anchors, cam)], axis=1)


def decode(anchors, mlp, books=None, idx=None, mask_logit=None, eps=0.01, cam=None):
    """Return float64 SoA Gaussians (mean, scale, quat, opacity, color) with
    n = na * k, Gaussian index a * k + i, plus the intermediates the adjoint
    uses.  cam: camera centre (3,) for the view-dependent input (W1 is then
    32 x 36), or None."""
    na, k = anchors.n, anchors.k
    f = mlp_input(anchors, cam)
    W1, b1 = np.asarray(mlp.W1, np.float64), np.asarray(mlp.b1, np.float64)
    W2, b2 = np.asarray(mlp.W2, np.float64), np.asarray(mlp.b2, np.float64)
    pre = f @ W1.T + b1
    h = np.maximum(pre, 0.0)
    y = (h @ W2.T + b2).reshape(na, k, OUT)
    opac = _sig(y[..., 0])
    color = _sig(y[..., 1:4])
    if books is None:
        logs = y[..., 4:7]
        quat = y[..., 7:11]
    else:
        v = np.zeros((na * k, 7))
        for s in range(books.shape[0]):
            v += np.asarray(books[s], np.float64)[idx[s]]
        logs = v[:, 0:3].reshape(na, k, 3)
        quat = v[:, 3:7].reshape(na, k, 4)
    scale = np.exp(logs)
    xa = np.asarray(anchors.xa, np.float64).T            # (na, 3)
    l = np.asarray(anchors.scaling, np.float64).T        # (na, 3)
    O = np.asarray(anchors.offset, np.float64)           # (na, k, 3)
    mean = xa[:, None, :] + O * l[:, None, :]
    keep = None
    if mask_logit is not None:
        keep = (_sig(np.asarray(mask_logit, np.float64)) > eps).reshape(na, k)
        opac = np.where(keep, opac, 0.0)
        scale = np.where(keep[..., None], scale, 0.0)
    n = na * k
    out = dict(mean=mean.reshape(n, 3).T.copy(), scale=scale.reshape(n, 3).T.copy(),
               quat=quat.reshape(n, 4).T.copy(), opacity=opac.reshape(n).copy(),
               color=color.reshape(n, 3).T.copy())
    out["_cache"] = dict(pre=pre, h=h, y=y, keep=keep, scale_raw=np.exp(logs).reshape(n, 3),
                         opac_raw=_sig(y[..., 0]).reshape(n))
    return out


def decode_backward(anchors, mlp, fwd, grads, books=None, idx=None, mask_logit=None, eps=0.01, cam=None):
    """Adjoint of ``decode``: from dL/d(mean, scale, quat, opacity, color)
    (float64 SoA) to dL/d(feat, W1, b1, W2, b2, offset, scaling, xa), the
    codebooks (row-wise segmented sums) and the mask logits; with a camera
    also dL/d(camera centre) ("cam"), and the view inputs' share of dL/dxa."""
    na, k = anchors.n, anchors.k
    n = na * k
    c = fwd["_cache"]
    dmean = np.asarray(grads["mean"], np.float64).T.reshape(na, k, 3)
    dscale = np.asarray(grads["scale"], np.float64).T.reshape(n, 3)
    dquat = np.asarray(grads["quat"], np.float64).T.reshape(n, 4)
    dop = np.asarray(grads["opacity"], np.float64).reshape(n)
    dcol = np.asarray(grads["color"], np.float64).T.reshape(n, 3)
    out = {}
    s_raw, o_raw = c["scale_raw"], c["opac_raw"]
    if mask_logit is not None:
        m = np.asarray(mask_logit, np.float64)
        keep = c["keep"].reshape(n)
        sg = _sig(m)
        # straight-through: d M / d m = sigmoid'(m); pruned Gaussians were culled and carry no gradient
        dM = (dscale * s_raw).sum(1) + dop * o_raw
        out["mask_logit"] = np.where(keep, sg * (1 - sg) * dM, 0.0)
        dscale = np.where(keep[:, None], dscale, 0.0)
        dop = np.where(keep, dop, 0.0)
    dy = np.zeros((n, OUT))
    y = c["y"].reshape(n, OUT)
    dy[:, 0] = dop * o_raw * (1 - o_raw)
    col = _sig(y[:, 1:4])
    dy[:, 1:4] = dcol * col * (1 - col)
    dlogs = dscale * s_raw
    if books is None:
        dy[:, 4:7] = dlogs
        dy[:, 7:11] = dquat
    else:
        dv = np.concatenate([dlogs, dquat], axis=1)
        out["books"] = []
        for s in range(books.shape[0]):
            db = np.zeros(books[s].shape)
            np.add.at(db, idx[s], dv)
            out["books"].append(db)
    dy = dy.reshape(na, k * OUT)
    W1, W2 = np.asarray(mlp.W1, np.float64), np.asarray(mlp.W2, np.float64)
    f = mlp_input(anchors, cam)
    out["W2"] = dy.T @ c["h"]
    out["b2"] = dy.sum(0)
    dh = dy @ W2
    dpre = dh * (c["pre"] > 0)
    out["W1"] = dpre.T @ f
    out["b1"] = dpre.sum(0)
    dx = dpre @ W1
    out["feat"] = dx[:, :32].copy()
    l = np.asarray(anchors.scaling, np.float64).T
    O = np.asarray(anchors.offset, np.float64)
    out["offset"] = dmean * l[:, None, :]
    out["scaling"] = (dmean * O).sum(1).T.copy()
    dxa = dmean.sum(1)
    if cam is not None:
        # delta = |v|, d = v / |v| with v = x_a - x_c:
        # dL/dv = dL/ddelta d + (dL/dd - (dL/dd . d) d) / delta
        vin = view_inputs(anchors, cam)
        delta, dirn = vin[:, 0], vin[:, 1:4]
        ddelta, ddir = dx[:, 32], dx[:, 33:36]
        dv = ddelta[:, None] * dirn + (ddir - (ddir * dirn).sum(1, keepdims=True) * dirn) / delta[:, None]
        dxa = dxa + dv
        out["cam"] = -dv.sum(0)
    out["xa"] = dxa.T.copy()
    return out


def pose_grad_from_centre(R, dcam):
    """dL/dxi (rho, phi) of the camera-centre path for the left perturbation
    exp(xi^) {R|t}: the centre c = -R^T t moves by -R^T rho to first order and
    not with phi, so dL/drho = -R dL/dc and dL/dphi = 0."""
    R = np.asarray(R, np.float64)
    return np.concatenate([-R @ np.asarray(dcam, np.float64), np.zeros(3)])
