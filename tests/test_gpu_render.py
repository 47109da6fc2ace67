"""GPU parity of the plain render path against the oracle, through the C ABI.

Bars: tile keys, sort order and tile ranges bit-exact; colour/depth/alpha
within 1e-4 absolute of the oracle on every pixel -- where a threshold decision
lies within FP32 noise (a flagged pixel), of one of the outcomes the oracle
enumerates for that pixel; A + T_final = 1 to the rounding of the sums;
gradients within 1e-3 relative per tensor (L2) and element by element
(|d| <= 1e-3 |g| + 1e-6 max|g|), the oracle following at each flagged pixel the
outcome the GPU took (zero upstream gradient only where two outcomes match).
"""
import numpy as np
import pytest
import torch

from oracle import raster
from paper_2403_11247_amd import scenes
from tests.gpu_common import (GRAD_REL_TOL, IMG_TOL, FIELDS, compare_images, compare_keys, dev, gauss_dev,
                              grad_check, rel_err, say, zero_at)

U32 = 2.0 ** -24

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    assert torch.cuda.is_available()
    vcgs.lib()
    return vcgs


def run_fwd(V, g, cam, pose, bg=(0.0, 0.0, 0.0)):
    gd = gauss_dev(g)
    C, D, A, st = V.render_forward(*gd, cam, pose, bg)
    torch.cuda.synchronize()
    return gd, C, D, A, st


def check_invariant(A, T, nc):
    """A + T_final = 1 per pixel, up to four roundings (of quantities <= 1) per
    contributor: the weight, the alpha sum, and the transmittance update."""
    A = A.cpu().numpy().astype(np.float64)
    T = T.cpu().numpy().astype(np.float64)
    nc = nc.cpu().numpy().astype(np.float64)
    dev_ = np.abs(A + T - 1.0)
    bound = 4.0 * U32 * (nc + 1.0)
    say("A + T_final - 1: max %.2e (bound at that pixel %.2e), %d pixels above 2e-6" %
        (dev_.max(initial=0.0), bound.ravel()[np.argmax(dev_)] if dev_.size else 0.0, int((dev_ > 2e-6).sum())))
    assert (dev_ <= bound).all()


def check_forward(V, g, cam, pose, bg=(0.0, 0.0, 0.0), name=""):
    say("forward", name, "n =", g.n, "image", cam.width, "x", cam.height)
    gd, C, D, A, st = run_fwd(V, g, cam, pose, bg)
    ref = raster.render(g, cam, pose, bg)
    compare_keys(st.view(), ref, g.n, cam)
    T, nc = st.pixel_state(cam.width, cam.height)
    r = compare_images(C, D, A, ref, g=g, cam=cam, pix_state=(T, nc))
    say(name, "max err colour %.2e depth %.2e alpha %.2e flagged %d (unmatched %d, ambiguous %d)" %
        (r["color"], r["depth"], r["alpha"], r["flagged"], r["flagged_unmatched"], r["flagged_ambiguous"]))
    assert r["pass_"], r
    check_invariant(A, T, nc)
    return gd, C, D, A, st, ref


def test_random_scene_forward(V):
    g = scenes.random_scene(2000, seed=0)
    check_forward(V, g, scenes.random_camera(), scenes.identity_pose(), name="random-2000")


@pytest.mark.parametrize("seed", [1, 2])
def test_random_scene_forward_posed(V, seed):
    rng = np.random.default_rng(seed)
    g = scenes.random_scene(3000, seed=seed, xy=1.5, log_scale=(0.005, 0.2))
    pose = scenes.perturb_pose(scenes.identity_pose(), seed, trans=0.3, rot_deg=10.0)
    check_forward(V, g, scenes.random_camera(), pose, bg=tuple(rng.uniform(0, 1, 3)), name=f"posed-{seed}")


def test_ragged_image_and_tiny_images(V):
    g = scenes.random_scene(500, seed=4)
    for (w, h) in [(100, 70), (17, 33), (1, 1), (16, 16), (257, 9)]:
        cam = scenes.Camera(w, h, 100.0 * w / 128, 100.0 * w / 128, w / 2.0, h / 2.0)
        check_forward(V, g, cam, scenes.identity_pose(), bg=(0.1, 0.2, 0.3), name=f"{w}x{h}")


def test_empty_and_all_culled(V):
    cam = scenes.random_camera()
    g0 = scenes.random_scene(0, seed=0)
    gd, C, D, A, st = run_fwd(V, g0, cam, scenes.identity_pose(), (0.2, 0.4, 0.6))
    assert torch.all(C[1] == np.float32(0.4)) and torch.all(A == 0) and torch.all(D == 0)
    up0 = [dev(x) for x in scenes.upstream_grads(cam.width, cam.height, seed=4)]
    _, dpose0 = V.render_backward(st, *gd, cam, scenes.identity_pose(), *up0)
    torch.cuda.synchronize()
    assert bool((dpose0 == 0).all())
    g = scenes.random_scene(100, seed=0)
    g.mean[2] = -1.0  # all behind the camera
    gd, C, D, A, st = run_fwd(V, g, cam, scenes.identity_pose(), (0.2, 0.4, 0.6))
    assert st.view()["n_pairs"] == 0 and torch.all(A == 0)
    # the backward of a map nothing of which is drawn: zero gradients, zero pose gradient
    up = [dev(x) for x in scenes.upstream_grads(cam.width, cam.height, seed=3)]
    grads, dpose = V.render_backward(st, *gd, cam, scenes.identity_pose(), *up)
    torch.cuda.synchronize()
    assert all(bool((grads[k] == 0).all()) for k in FIELDS) and bool((dpose == 0).all())


def test_depth_ties_keep_index_order(V):
    g = scenes.random_scene(600, seed=5)
    g.mean[:, 300:600] = g.mean[:, 0:300]
    check_forward(V, g, scenes.random_camera(), scenes.identity_pose(), name="ties")


@pytest.mark.parametrize("n", [6000, 20000])
def test_long_tile_lists_keep_the_oracle_order(V, n):
    """Every one of the 12 tiles of a 64x48 view holds about n entries (6000,
    20000): long per-tile lists, each in (depth, index) order.  Depths are
    rounded to 1 cm so that many entries tie."""
    rng = np.random.default_rng(n)
    mean = np.stack([rng.uniform(-0.1, 0.1, n), rng.uniform(-0.08, 0.08, n), np.round(rng.uniform(2.0, 3.0, n), 2)])
    g = scenes.Gaussians(mean.astype(np.float32), np.full((3, n), 0.45, np.float32),
                         rng.normal(size=(4, n)).astype(np.float32), rng.uniform(0.05, 0.6, n).astype(np.float32),
                         rng.uniform(0, 1, (3, n)).astype(np.float32))
    cam = scenes.Camera(64, 48, 40.0, 40.0, 32.0, 24.0)
    gd, C, D, A, st, ref = check_forward(V, g, cam, scenes.identity_pose(), name=f"long-{n}")
    rng_ = ref["ranges"]
    assert int((rng_[:, 1] - rng_[:, 0]).min()) > 0.9 * n, rng_


def test_forward_is_deterministic(V):
    g = scenes.random_scene(2000, seed=3)
    cam = scenes.random_camera()
    _, C1, D1, A1, s1 = run_fwd(V, g, cam, scenes.identity_pose())
    _, C2, D2, A2, s2 = run_fwd(V, g, cam, scenes.identity_pose())
    assert torch.equal(C1, C2) and torch.equal(D1, D2) and torch.equal(A1, A2)
    assert torch.equal(s1.view()["gids"], s2.view()["gids"])


def check_backward(V, g, cam, pose, up, bg=(0.0, 0.0, 0.0), name="", tol=GRAD_REL_TOL):
    gd, C, D, A, st = run_fwd(V, g, cam, pose, bg)
    ref = raster.render(g, cam, pose, bg)
    r = compare_images(C, D, A, ref, g=g, cam=cam, pix_state=st.pixel_state(cam.width, cam.height))
    assert r["pass_"], r
    # the oracle follows the outcome the GPU took at each flagged pixel; where
    # that is not unique, or the 0.99 clamp is ambiguous, the pixel gets no gradient
    skip = (r["variant"] < 0) | ((ref["flags"] & 4) != 0)
    up = zero_at(up, skip)
    say("backward", name, "flagged", r["flagged"], "without gradient", int(skip.sum()))
    grads, dpose = V.render_backward(st, *gd, cam, pose, dev(up[0]), dev(up[1]), dev(up[2]))
    torch.cuda.synchronize()
    gref = raster.render_backward(g, cam, pose, ref, *up, variant=np.maximum(r["variant"], 0))
    errs = {}
    for k in FIELDS:
        errs[k] = grad_check(k, grads[k].cpu().numpy(), gref[k], tol)
    errs["pose"] = grad_check("pose", dpose.cpu().numpy(), gref["pose"], tol)
    say(name, "grad rel err", {k: "%.2e" % v for k, v in errs.items()})
    return grads, dpose, gref


def test_random_scene_backward(V):
    g = scenes.random_scene(2000, seed=0)
    cam = scenes.random_camera()
    up = scenes.upstream_grads(cam.width, cam.height, seed=1)
    check_backward(V, g, cam, scenes.identity_pose(), up, name="random-2000")


def test_posed_backward_with_background(V):
    g = scenes.random_scene(1500, seed=7, xy=1.5, log_scale=(0.01, 0.1))
    pose = scenes.perturb_pose(scenes.identity_pose(), 3, trans=0.2, rot_deg=8.0)
    cam = scenes.Camera(96, 80, 80.0, 85.0, 50.0, 38.0)
    up = scenes.upstream_grads(cam.width, cam.height, seed=4)
    check_backward(V, g, cam, pose, up, bg=(0.3, 0.6, 0.9), name="posed-bg")


@pytest.mark.parametrize("H,W", [(20, 30), (19, 31), (68, 120), (67, 121)])
def test_l1_loss_kernel(V, H, W):
    # pixel counts divisible by 4 take the 4-pixel vector path, the others one pixel per thread;
    # equal values (zero error, zero gradient) in every other row
    rng = np.random.default_rng(0)
    C = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    D = rng.uniform(1, 5, (H, W)).astype(np.float32)
    Ct, Dt = C.copy(), D.copy()
    Ct[:, ::2] += 0.1
    Dt[1::3] -= 0.2
    loss, dlc, dld = V.l1_loss(dev(C), dev(D), dev(Ct), dev(Dt), 0.5)
    n = H * W
    exp_loss = (np.abs(C.astype(np.float64) - Ct).sum() + 0.5 * np.abs(D.astype(np.float64) - Dt).sum()) / n
    assert abs(float(loss.cpu()) - exp_loss) < 1e-5 * exp_loss
    np.testing.assert_array_equal(dlc.cpu().numpy(), (np.sign(C - Ct) / np.float32(n)).astype(np.float32))
    np.testing.assert_allclose(dld.cpu().numpy(), 0.5 * np.sign(D - Dt) / n, rtol=1e-6)
