"""Pins of the tracking/BA loss oracle (Sec. 3.5 eqs. (19)-(21), SSIM for BA)
against what the mathematics fixes: closed forms for constant errors and a
shifted plane, the silhouette indicator and the depth validity as exact
selections, k-d tree nearest neighbours, scipy's zero-padded correlation, the
SSIM of constant images, symmetry and identity, and finite differences of every
gradient (colour, depth, Gaussian centres, pose under the left perturbation,
SSIM)."""
import math

import numpy as np
import pytest
from scipy import ndimage
from scipy.spatial import cKDTree

from oracle import track
from paper_2403_11247_amd import scenes


def _imgs(rng, H=12, W=17):
    C = rng.uniform(0, 1, (3, H, W))
    tC = rng.uniform(0, 1, (3, H, W))
    D = rng.uniform(1, 3, (H, W))
    tD = rng.uniform(1, 3, (H, W))
    tD[rng.uniform(size=(H, W)) < 0.2] = 0.0
    A = rng.uniform(0.9, 1.0, (H, W))
    return C, D, A, tC, tD


def test_track_loss_constant_errors_closed_form():
    H, W = 8, 10
    C = np.full((3, H, W), 0.5)
    tC = C - 0.1
    D = np.full((H, W), 2.0)
    tD = D - 0.2
    tD[0, :] = 0.0  # no observation on the first row
    A = np.ones((H, W))
    for norm, (lc, ld) in ((2, (3 * 0.01, 0.04)), (1, (3 * 0.1, 0.2))):
        loss, _, _ = track.track_loss(C, D, A, tC, tD, lam_d=0.5, norm=norm)
        assert loss == pytest.approx(lc + 0.5 * ld, rel=1e-12)


@pytest.mark.parametrize("norm", [1, 2])
def test_track_loss_selection_and_gradient(norm):
    rng = np.random.default_rng(norm)
    C, D, A, tC, tD = _imgs(rng)
    loss, gC, gD = track.track_loss(C, D, A, tC, tD, lam_d=0.7, norm=norm)
    off = A <= 0.99
    assert off.any() and np.all(gC[:, off] == 0) and np.all(gD[off] == 0)
    assert np.all(gD[tD == 0] == 0)
    h = 1e-6
    for _ in range(20):
        c, i, j = rng.integers(0, 3), rng.integers(0, C.shape[1]), rng.integers(0, C.shape[2])
        Cp, Cm = C.copy(), C.copy()
        Cp[c, i, j] += h
        Cm[c, i, j] -= h
        fd = (track.track_loss(Cp, D, A, tC, tD, 0.7, norm)[0] - track.track_loss(Cm, D, A, tC, tD, 0.7, norm)[0]) / (2 * h)
        assert fd == pytest.approx(gC[c, i, j], rel=1e-6, abs=1e-9)
        Dp, Dm = D.copy(), D.copy()
        Dp[i, j] += h
        Dm[i, j] -= h
        fd = (track.track_loss(C, Dp, A, tC, tD, 0.7, norm)[0] - track.track_loss(C, Dm, A, tC, tD, 0.7, norm)[0]) / (2 * h)
        assert fd == pytest.approx(gD[i, j], rel=1e-6, abs=1e-9)


def _plane_case(stride=1, H=30, W=40, z=2.0):
    cam = scenes.Camera(W, H, 40.0, 40.0, W / 2, H / 2)
    depth = np.full((H, W), z)
    depth[3:6, 4:9] = 0.0
    return cam, depth


def test_icp_nearest_neighbours_match_kdtree():
    rng = np.random.default_rng(3)
    cam = scenes.Camera(40, 30, 35.0, 35.0, 20.0, 15.0)
    depth = rng.uniform(1.0, 3.0, (30, 40))
    depth[rng.uniform(size=depth.shape) < 0.1] = 0.0
    pose = scenes.perturb_pose(scenes.identity_pose(), 4, trans=0.05, rot_deg=3.0)
    means = rng.uniform([-1, -1, 1], [1, 1, 3], (300, 3)).T
    for stride in (1, 3):
        out = track.icp(means, pose, depth, cam, tau=0.2, stride=stride)
        R = np.asarray(pose.R, np.float64).reshape(3, 3)
        pc = (R @ means).T + np.asarray(pose.t, np.float64)
        dist, _ = cKDTree(out["pts"]).query(pc)
        np.testing.assert_allclose(out["dist"], dist, rtol=1e-12)
        assert out["w"].sum() > 10


def test_backprojection_lands_on_pixel_centres():
    """Projecting the back-projected points with the pinhole model gives the
    pixel centres (u + 0.5, v + 0.5) and the observed depths."""
    rng = np.random.default_rng(13)
    cam = scenes.Camera(37, 23, 31.0, 29.0, 17.3, 12.1)
    depth = rng.uniform(0.5, 4.0, (23, 37))
    depth[rng.uniform(size=depth.shape) < 0.3] = 0.0
    for stride in (1, 2, 5):
        pts = track.backproject(depth, cam, stride)
        v, u = np.nonzero(depth[::stride, ::stride] > 0)
        np.testing.assert_allclose(cam.fx * pts[:, 0] / pts[:, 2] + cam.cx, u * stride + 0.5, rtol=0, atol=1e-9)
        np.testing.assert_allclose(cam.fy * pts[:, 1] / pts[:, 2] + cam.cy, v * stride + 0.5, rtol=0, atol=1e-9)
        np.testing.assert_allclose(pts[:, 2], depth[::stride, ::stride][v, u], rtol=1e-15)


def test_icp_weights_are_the_tau_test_on_kdtree_distances():
    rng = np.random.default_rng(14)
    cam = scenes.Camera(40, 30, 35.0, 35.0, 20.0, 15.0)
    depth = rng.uniform(1.0, 3.0, (30, 40))
    means = rng.uniform([-1, -1, 1], [1, 1, 3], (500, 3)).T
    for tau in (0.03, 0.1, 0.3):
        out = track.icp(means, scenes.identity_pose(), depth, cam, tau)
        dist, _ = cKDTree(out["pts"]).query(means.T)
        assert np.array_equal(out["w"] > 0, dist < tau)
        assert 0 < out["w"].sum() < means.shape[1]


def test_icp_shifted_plane_closed_form():
    cam, depth = _plane_case()
    pts = track.backproject(depth, cam)
    delta = 0.01
    means = (pts + np.array([0.0, 0.0, delta])).T
    out = track.icp(means, scenes.identity_pose(), depth, cam, tau=0.05)
    n = pts.shape[0]
    assert np.all(out["w"] == 1)
    assert out["loss"] == pytest.approx(n * delta ** 2, rel=1e-9)
    np.testing.assert_allclose(out["dpose"][:3], [0, 0, 2 * n * delta], atol=1e-9)
    exact = track.icp(pts.T, scenes.identity_pose(), depth, cam, tau=0.05)
    assert exact["loss"] == 0.0


def test_icp_gradients_by_finite_differences():
    rng = np.random.default_rng(5)
    cam = scenes.Camera(40, 30, 35.0, 35.0, 20.0, 15.0)
    depth = rng.uniform(1.5, 2.5, (30, 40))
    pose = scenes.perturb_pose(scenes.identity_pose(), 6, trans=0.03, rot_deg=2.0)
    means = (track.backproject(depth, cam)[rng.integers(0, 1200, 200)] + rng.normal(0, 0.02, (200, 3))).T
    base = track.icp(means, pose, depth, cam, tau=0.1)
    assert base["w"].sum() > 50
    R = np.asarray(pose.R, np.float64).reshape(3, 3)
    t = np.asarray(pose.t, np.float64)
    h = 1e-7

    def loss_at(xi):
        rho, phi = xi[:3], xi[3:]
        th = np.linalg.norm(phi)
        K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
        E = np.eye(3) + (math.sin(th) / th if th else 1.0) * K + ((1 - math.cos(th)) / th ** 2 if th else 0.5) * K @ K
        p2 = scenes.Pose(E @ R, E @ t + rho)
        o = track.icp(means, p2, depth, cam, tau=0.1)
        assert np.array_equal(o["nn"], base["nn"]) and np.array_equal(o["w"], base["w"])
        return o["loss"]

    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        fd = (loss_at(e) - loss_at(-e)) / (2 * h)
        assert fd == pytest.approx(base["dpose"][k], rel=1e-5, abs=1e-7)
    for i in np.nonzero(base["w"])[0][:5]:
        for a in range(3):
            mp, mm = means.copy(), means.copy()
            mp[a, i] += h
            mm[a, i] -= h
            fd = (track.icp(mp, pose, depth, cam, 0.1)["loss"] - track.icp(mm, pose, depth, cam, 0.1)["loss"]) / (2 * h)
            assert fd == pytest.approx(base["dmeans"][a, i], rel=1e-5, abs=1e-7)


def test_filter_is_zero_padded_correlation():
    rng = np.random.default_rng(7)
    img = rng.normal(size=(23, 31))
    g = track.gauss_window()
    ref = ndimage.correlate(img, np.outer(g, g), mode="constant", cval=0.0)
    np.testing.assert_allclose(track._filt(img, g), ref, rtol=1e-12, atol=1e-14)
    assert g.sum() == pytest.approx(1.0) and g[5] == g.max() and np.allclose(g, g[::-1])


def test_ssim_closed_forms_and_symmetry():
    H, W = 30, 33
    a, b = 0.3, 0.6
    x = np.full((3, H, W), a)
    y = np.full((3, H, W), b)
    _, _, m = track.ssim(x, y)
    inner = m[:, 5:-5, 5:-5]
    np.testing.assert_allclose(inner, (2 * a * b + track.C1) / (a * a + b * b + track.C1), rtol=1e-12)
    rng = np.random.default_rng(8)
    x = rng.uniform(0, 1, (3, H, W))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    l_xy, g, _ = track.ssim(x, y)
    l_yx, _, _ = track.ssim(y, x)
    assert l_xy == pytest.approx(l_yx, rel=1e-12)
    l_xx, g_xx, _ = track.ssim(x, x)
    assert abs(l_xx) < 1e-12 and np.abs(g_xx).max() < 1e-12
    assert 0.0 < l_xy < 1.0


def test_ssim_gradient_by_finite_differences():
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 1, (3, 16, 19))
    y = rng.uniform(0, 1, (3, 16, 19))
    _, g, _ = track.ssim(x, y)
    h = 1e-6
    for _ in range(25):
        c, i, j = rng.integers(0, 3), rng.integers(0, 16), rng.integers(0, 19)
        xp, xm = x.copy(), x.copy()
        xp[c, i, j] += h
        xm[c, i, j] -= h
        fd = (track.ssim(xp, y)[0] - track.ssim(xm, y)[0]) / (2 * h)
        assert fd == pytest.approx(g[c, i, j], rel=1e-5, abs=1e-10)
