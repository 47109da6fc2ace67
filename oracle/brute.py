"""Brute-force renderer: the definition, with no tiles and no sort keys.

Test infrastructure only.  Every pixel composites every Gaussian, nearest
first (camera depth, ties by index), with the footprint of eq. (1) under the
projection of eqs. (2)-(3), and the sums of eqs. (16)-(18).  Written with
plain PyTorch CPU ops in float64 so that the same code gives values and, under
autograd, gradients that do not depend on the hand-derived adjoint in raster.c.

Readings shared with the rest of the oracle (the paper is silent on them):
pixel centres at half-integers; footprint min(0.99, o exp(power)) skipped
below 1/255; the Gaussian that would take the transmittance under 1e-4 is
excluded and the pixel stops; depth = camera z of the mean; x/z and y/z
clamped to 1.3 x half-extent / focal length inside J; 0.3 added to the
diagonal of Sigma'; pose perturbed on the left by exp(xi^), xi = (rho, phi).
"""
from __future__ import annotations

import numpy as np
import torch

F32 = np.float32
ALPHA_MIN = float(F32(1.0) / F32(255.0))
ALPHA_MAX = float(F32(0.99))
T_MIN = float(F32(1e-4))
LOWPASS = float(F32(0.3))
CLAMP_FOV = float(F32(1.3))


def _skew(v):
    z = torch.zeros((), dtype=v.dtype)
    return torch.stack([torch.stack([z, -v[2], v[1]]),
                        torch.stack([v[2], z, -v[0]]),
                        torch.stack([-v[1], v[0], z])])


def quat_to_rot(q):
    """Rotation of the normalised quaternion (w, x, y, z); q has shape (4, n)."""
    n2 = (q * q).sum(0)
    safe = n2 > 0
    qn = torch.where(safe, torch.sqrt(torch.where(safe, n2, torch.ones_like(n2))), torch.ones_like(n2))
    unit = torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=q.dtype)[:, None]
    qh = torch.where(safe[None, :], q / qn[None, :], unit)
    w, x, y, z = qh
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]),
    ])  # (3, 3, n)


def project(mean, scale, quat, cam, R, t):
    """Camera point (3,n), 2D mean (u, v), inverse 2D covariance (n,2,2)."""
    pc = R @ mean + t[:, None]
    X, Y, Z = pc
    Rq = quat_to_rot(quat)
    M = Rq * scale[None, :, :]                       # M_ij = r_ij s_j
    Sig = torch.einsum("ikn,jkn->nij", M, M)         # eq. (2): R S S^T R^T
    limx = CLAMP_FOV * (0.5 * cam.width / cam.fx)
    limy = CLAMP_FOV * (0.5 * cam.height / cam.fy)
    xz = torch.clamp(X / Z, -limx, limx)
    yz = torch.clamp(Y / Z, -limy, limy)
    zero = torch.zeros_like(Z)
    J = torch.stack([torch.stack([cam.fx / Z, zero, -cam.fx * xz / Z]),
                     torch.stack([zero, cam.fy / Z, -cam.fy * yz / Z])]).permute(2, 0, 1)  # (n,2,3)
    JW = J @ R                                      # eq. (3): J W
    Sp = JW @ Sig @ JW.transpose(1, 2) + LOWPASS * torch.eye(2, dtype=mean.dtype)
    Q = torch.linalg.inv(Sp)
    u = cam.fx * X / Z + cam.cx
    v = cam.fy * Y / Z + cam.cy
    return pc, u, v, Q


def render(mean, scale, quat, opacity, color, cam, R, t, bg=(0.0, 0.0, 0.0), xi=None, hits=None):
    """Brute-force render; every input a float64 tensor (SoA shapes as in
    the ABI).  ``xi`` (6,) perturbs the pose on the left.  Returns
    (C (3,H,W), D (H,W), A (H,W), T_final (H,W)).  ``hits`` (numpy, n) if
    given receives each Gaussian's number of blended pixels (eq. (13), h)."""
    if xi is not None:
        E = torch.matrix_exp(_skew(xi[3:6]))
        R = E @ R
        t = E @ t + xi[0:3]
    pc, u, v, Q = project(mean, scale, quat, cam, R, t)
    Z = pc[2]
    W, H = cam.width, cam.height
    ys, xs = torch.meshgrid(torch.arange(H, dtype=mean.dtype) + 0.5,
                            torch.arange(W, dtype=mean.dtype) + 0.5, indexing="ij")
    px, py = xs.reshape(-1), ys.reshape(-1)
    vis = (Z.detach() > cam.z_near) & (opacity.detach() >= ALPHA_MIN)
    idx = [i for i in range(mean.shape[1]) if bool(vis[i])]
    idx.sort(key=lambda i: (float(Z[i].detach()), i))
    T = torch.ones(H * W, dtype=mean.dtype)
    Cc = torch.zeros((3, H * W), dtype=mean.dtype)
    D = torch.zeros(H * W, dtype=mean.dtype)
    A = torch.zeros(H * W, dtype=mean.dtype)
    done = torch.zeros(H * W, dtype=torch.bool)
    for i in idx:
        dx, dy = px - u[i], py - v[i]
        power = -0.5 * (Q[i, 0, 0] * dx * dx + Q[i, 1, 1] * dy * dy) - Q[i, 0, 1] * dx * dy
        raw = opacity[i] * torch.exp(power)                       # eq. (1) on the image plane
        alpha = torch.where(raw > ALPHA_MAX, torch.full_like(raw, ALPHA_MAX), raw)
        valid = (alpha.detach() >= ALPHA_MIN) & ~done
        Tn = T * (1 - alpha)
        stop = valid & (Tn.detach() < T_MIN)
        take = valid & ~stop
        w = torch.where(take, alpha * T, torch.zeros_like(T))
        if hits is not None:
            hits[i] = int(take.sum())
        Cc = Cc + w[None, :] * color[:, i:i + 1]                  # eq. (16)
        D = D + w * Z[i]                                          # eq. (17)
        A = A + w                                                 # eq. (18)
        T = torch.where(take, Tn, T)
        done = done | stop
    bgv = torch.as_tensor(bg, dtype=mean.dtype)
    Cc = Cc + T[None, :] * bgv[:, None]
    return Cc.reshape(3, H, W), D.reshape(H, W), A.reshape(H, W), T.reshape(H, W)


def as64(g):
    """float64 leaf tensors of a scenes.Gaussians."""
    return [torch.tensor(np.asarray(a, np.float64), requires_grad=True)
            for a in (g.mean, g.scale, g.quat, g.opacity, g.color)]


def render_np(g, cam, pose, bg=(0.0, 0.0, 0.0)):
    """numpy convenience wrapper: float64 arrays (C, D, A, T_final)."""
    with torch.no_grad():
        ts = [torch.tensor(np.asarray(a, np.float64)) for a in (g.mean, g.scale, g.quat, g.opacity, g.color)]
        out = render(*ts, cam, torch.tensor(pose.R, dtype=torch.float64),
                     torch.tensor(pose.t, dtype=torch.float64), bg)
    return [o.numpy() for o in out]


def grads(g, cam, pose, dl_dc, dl_dd, dl_da, bg=(0.0, 0.0, 0.0)):
    """Autograd gradients of sum(dl_dc*C + dl_dd*D + dl_da*A) with respect to
    every Gaussian attribute and the pose tangent xi = (rho, phi) at 0."""
    ts = as64(g)
    xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    C, D, A, _ = render(*ts, cam, torch.tensor(pose.R, dtype=torch.float64),
                        torch.tensor(pose.t, dtype=torch.float64), bg, xi=xi)
    L = (torch.as_tensor(dl_dc, dtype=torch.float64) * C).sum() \
        + (torch.as_tensor(dl_dd, dtype=torch.float64) * D).sum() \
        + (torch.as_tensor(dl_da, dtype=torch.float64) * A).sum()
    L.backward()
    out = {k: v.grad.numpy() for k, v in zip(("mean", "scale", "quat", "opacity", "color"), ts)}
    out["pose"] = xi.grad.numpy()
    return out


def loss_value(g64, cam, pose, dl_dc, dl_dd, dl_da, xi=None, bg=(0.0, 0.0, 0.0)):
    """Scalar sum(dl_dc*C + dl_dd*D + dl_da*A) for float64 numpy inputs
    (used by finite differences)."""
    with torch.no_grad():
        ts = [torch.tensor(np.asarray(a, np.float64)) for a in g64]
        C, D, A, _ = render(*ts, cam, torch.tensor(np.asarray(pose.R, np.float64)),
                            torch.tensor(np.asarray(pose.t, np.float64)), bg,
                            xi=None if xi is None else torch.tensor(xi, dtype=torch.float64))
        return float((torch.as_tensor(dl_dc) * C).sum() + (torch.as_tensor(dl_dd) * D).sum()
                     + (torch.as_tensor(dl_da) * A).sum())
