"""Tracking on top of the renderer (Sec. 3.5 eq. (21)): starting 3 cm and
1.5 degrees off, repeated iterations of render, silhouette-masked L1 colour
and depth loss, backward to the pose, and the ICP term's pose gradient, with
Adam steps on the left perturbation, bring the pose back toward the one the
observed frame was rendered from."""
import math

import numpy as np
import pytest
import torch

from paper_2403_11247_amd import scenes
from tests.gpu_common import FIELDS, gauss_dev, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    vcgs.lib()
    return vcgs


def _expm(xi):
    rho, phi = xi[:3], xi[3:]
    th = np.linalg.norm(phi)
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    E = np.eye(3) + (math.sin(th) / th if th else 1.0) * K + ((1 - math.cos(th)) / th ** 2 if th else 0.5) * K @ K
    return E, rho


def _pose_error(p, ref):
    R, t = np.asarray(p.R, np.float64), np.asarray(p.t, np.float64)
    R0, t0 = np.asarray(ref.R, np.float64), np.asarray(ref.t, np.float64)
    dR = R @ R0.T
    ang = math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(dR) - 1) / 2))))
    return float(np.linalg.norm(-R.T @ t + R0.T @ t0)), ang


def test_tracking_iterations_recover_the_pose(V):
    from oracle import decode as odec
    a = scenes.room_anchors(10000, k=10, seed=3)
    m = scenes.room_mlp(seed=3)
    d = odec.decode(a, m)
    g = scenes.Gaussians(*[d[f].astype(np.float32) for f in FIELDS])
    gd = gauss_dev(g)
    cam = scenes.Camera(320, 180, 160.0, 160.0, 160.0, 90.0)
    _, true_pose = scenes.room_camera()
    tC, tD, tA, _ = V.render_forward(*gd, cam, true_pose, keep_state=False)
    obs = torch.where(tA >= 0.5, tD / tA.clamp_min(0.5), torch.zeros_like(tD))
    cur = scenes.perturb_pose(true_pose, 9, trans=0.03, rot_deg=1.5)
    e0 = _pose_error(cur, true_pose)
    lr = np.array([2e-3] * 3 + [1e-3] * 3)
    mo, ve = np.zeros(6), np.zeros(6)
    first = last = None
    for it in range(1, 61):
        C, D, A, st = V.render_forward(*gd, cam, cur)
        loss, dlc, dld = V.track_loss(C, D, A, tC, obs, lam_d=1.0, norm=1)
        _, dpose = V.render_backward(st, *gd, cam, cur, dlc, dld, None)
        V.icp_loss(gd[0], cam, cur, obs, tau=0.05, stride=2, weight=1e-4, dpose=dpose)
        st.free()
        gxi = dpose.double().cpu().numpy()
        lv = float(loss[0])
        first = lv if first is None else first
        last = lv
        mo = 0.9 * mo + 0.1 * gxi
        ve = 0.999 * ve + 0.001 * gxi ** 2
        step = -lr * (mo / (1 - 0.9 ** it)) / (np.sqrt(ve / (1 - 0.999 ** it)) + 1e-12)
        E, rho = _expm(step)
        cur = scenes.Pose((E @ np.asarray(cur.R, np.float64)).astype(np.float32),
                          (E @ np.asarray(cur.t, np.float64) + rho).astype(np.float32))
    e1 = _pose_error(cur, true_pose)
    say(f"tracking: loss {first:.4f} -> {last:.4f}; centre {e0[0] * 100:.2f} -> {e1[0] * 100:.2f} cm, "
        f"rotation {e0[1]:.3f} -> {e1[1]:.3f} deg")
    assert last < 0.3 * first
    assert e1[1] < 0.5 * e0[1]
    assert e1[0] < 0.8 * e0[0]
