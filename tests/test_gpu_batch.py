"""Batched views (vcgs_render_batch): a bundle-adjustment window of mixed-size
views of one map, in one pass, eagerly or as a replayed hipGraph.

Bars: images bitwise equal to per-view plain calls (the same per-tile lists
in the same order, the same arithmetic); pose gradients and per-view losses
within 1e-5 relative; Gaussian gradients (summed over the views in a fixed
order instead of by the caller) within 1e-5 relative; each view within 1e-4 of
the oracle on unflagged pixels."""
import numpy as np
import pytest
import torch

from oracle import raster
from paper_2403_11247_amd import scenes
from tests.gpu_common import FIELDS, compare_images, dev, gauss_dev, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    vcgs.lib()
    return vcgs


def small_window(n_views=5, seed=0):
    cams = [scenes.Camera(w, h, 0.8 * w, 0.8 * w, w / 2.0, h / 2.0)
            for (w, h) in [(64, 48), (100, 70), (128, 96), (33, 17), (80, 80), (48, 64)][:n_views]]
    base = scenes.identity_pose()
    poses = [scenes.perturb_pose(base, seed + i, trans=0.1, rot_deg=4.0) for i in range(n_views)]
    return cams, poses


def plain_views(V, gd, cams, poses, targets=None, w_depth=0.5):
    out = []
    for i, (c, p) in enumerate(zip(cams, poses)):
        C, D, A, st = V.render_forward(*gd, c, p)
        r = {"C": C, "D": D, "A": A}
        if targets is not None:
            loss, dlc, dld = V.l1_loss(C, D, targets[i][0], targets[i][1], w_depth)
            grads, dpose = V.render_backward(st, *gd, c, p, dlc, dld, None)
            r.update(loss=loss, grads=grads, dpose=dpose)
        st.free()
        out.append(r)
    torch.cuda.synchronize()
    return out


def random_targets(cams, seed=3):
    rng = np.random.default_rng(seed)
    return [(dev(rng.uniform(0, 1, (3, c.height, c.width))), dev(rng.uniform(1.5, 4.5, (c.height, c.width))))
            for c in cams]


def test_batch_forward_equals_plain_and_oracle(V):
    g = scenes.random_scene(3000, seed=2, xy=1.2)
    gd = gauss_dev(g)
    cams, poses = small_window()
    win = V.BatchWindow(g.n, cams, backward=False)
    win.run(*gd, poses)
    torch.cuda.synchronize()
    ref = plain_views(V, gd, cams, poses)
    for i, (c, p) in enumerate(zip(cams, poses)):
        C, D, A = win.outs[i]
        assert torch.equal(C, ref[i]["C"]) and torch.equal(D, ref[i]["D"]) and torch.equal(A, ref[i]["A"]), i
        r = compare_images(C, D, A, raster.render(g, c, p), g=g, cam=c)
        assert r["pass_"], (i, r)
    say("batch forward", len(cams), "views, pairs", win.pairs)


def check_backward(win, ref, V_=None):
    for i in range(win.V):
        C, D, A = win.outs[i]
        assert torch.equal(C, ref[i]["C"]), i
        assert abs(float(win.loss[i]) - float(ref[i]["loss"][0])) <= 1e-5 * abs(float(ref[i]["loss"][0])) + 1e-9
        e = rel_err(win.dpose[i].cpu().numpy(), ref[i]["dpose"].cpu().numpy())
        assert e <= 1e-5, (i, e)
    for k in FIELDS:
        tot = sum(r["grads"][k] for r in ref)
        e = rel_err(win.grads[k].cpu().numpy(), tot.cpu().numpy())
        assert e <= 1e-5, (k, e)


def test_batch_backward_equals_plain(V):
    g = scenes.random_scene(3000, seed=4, xy=1.2)
    gd = gauss_dev(g)
    cams, poses = small_window(seed=10)
    tg = random_targets(cams)
    win = V.BatchWindow(g.n, cams, backward=True)
    win.run(*gd, poses, tg)
    torch.cuda.synchronize()
    check_backward(win, plain_views(V, gd, cams, poses, tg))


def test_graph_replays_follow_new_poses(V):
    g = scenes.random_scene(3000, seed=5, xy=1.2)
    gd = gauss_dev(g)
    cams, _ = small_window(seed=20)
    tg = random_targets(cams, seed=6)
    win = V.BatchWindow(g.n, cams, backward=True, graph=True)
    for it in range(4):
        _, poses = small_window(seed=30 + it)
        win.run(*gd, poses, tg)
        torch.cuda.synchronize()
        say("graph replay", it, "pairs", win.pairs)
        check_backward(win, plain_views(V, gd, cams, poses, tg))


def test_capacity_overflow_is_reported_and_rerun(V):
    """A window first sized on distant poses is then rendered from close up:
    the pairs outgrow the buffers, the check reports it, the binding reruns."""
    g = scenes.random_scene(3000, seed=7, xy=1.0, log_scale=(0.05, 0.2))
    gd = gauss_dev(g)
    cams = [scenes.Camera(w, h, 0.8 * w, 0.8 * w, w / 2.0, h / 2.0) for (w, h) in [(200, 150), (160, 120), (240, 180)]]
    far = [scenes.Pose(np.eye(3, dtype=np.float32), np.array([0, 0, 20.0], np.float32))] * 3
    near = [scenes.Pose(np.eye(3, dtype=np.float32), np.array([0, 0, -1.2], np.float32))] * 3
    tg = random_targets(cams, seed=8)
    for graph in (False, True):
        win = V.BatchWindow(g.n, cams, backward=True, graph=graph)
        win.run(*gd, far, tg)
        small = win.pairs
        win.run(*gd, near, tg)
        torch.cuda.synchronize()
        assert win.pairs > small + small // 8 + 4096, (small, win.pairs)
        check_backward(win, plain_views(V, gd, cams, near, tg))


def test_ba_window_full_size(V):
    """12 keyframes (4 x 320x240, 4 x 640x480, 4 x 1200x680) of a 500k-Gaussian room."""
    from oracle import decode as odec
    a = scenes.room_anchors(50000, k=10, seed=1)
    m = scenes.room_mlp(seed=1)
    dec = odec.decode(a, m)
    g = scenes.Gaussians(*[dec[f].astype(np.float32) for f in FIELDS])
    gd = gauss_dev(g)
    cams, poses = scenes.ba_window(12)
    tposes = [scenes.perturb_pose(p, 100 + i) for i, p in enumerate(poses)]
    tg = []
    for c, p in zip(cams, tposes):
        C, D, A, _ = V.render_forward(*gd, c, p, keep_state=False)
        tg.append((C, D))
    win = V.BatchWindow(g.n, cams, backward=True, graph=True)
    win.run(*gd, poses, tg)
    torch.cuda.synchronize()
    say("BA window pairs", win.pairs)
    check_backward(win, plain_views(V, gd, cams, poses, tg))
    # one full-size view against the oracle
    i = 8
    r = compare_images(*win.outs[i], raster.render(g, cams[i], poses[i]), g=g, cam=cams[i])
    say("BA view", i, "max err colour %.2e depth %.2e flagged %d" % (r["color"], r["depth"], r["flagged"]))
    assert r["pass_"], r


def test_unchecked_passes_then_one_check(V):
    """Passes enqueued back to back without a host synchronisation (eager and
    graph windows, the graph launched on the caller's stream), then one check:
    the last pass's results equal the plain calls, and a window whose pairs
    outgrow its buffers while unchecked is reported by the later check."""
    g = scenes.random_scene(3000, seed=9, xy=1.2)
    gd = gauss_dev(g)
    cams, _ = small_window(seed=40)
    tg = random_targets(cams, seed=10)
    for graph in (False, True):
        win = V.BatchWindow(g.n, cams, backward=True, graph=graph)
        for it in range(3):
            _, poses = small_window(seed=41 + it)
            win.run(*gd, poses, tg, check=False)
        assert win.check()
        check_backward(win, plain_views(V, gd, cams, poses, tg))
    g2 = scenes.random_scene(3000, seed=7, xy=1.0, log_scale=(0.05, 0.2))
    gd2 = gauss_dev(g2)
    cams2 = [scenes.Camera(w, h, 0.8 * w, 0.8 * w, w / 2.0, h / 2.0) for (w, h) in [(200, 150), (160, 120)]]
    far = [scenes.Pose(np.eye(3, dtype=np.float32), np.array([0, 0, 20.0], np.float32))] * 2
    near = [scenes.Pose(np.eye(3, dtype=np.float32), np.array([0, 0, -1.2], np.float32))] * 2
    tg2 = random_targets(cams2, seed=11)
    win = V.BatchWindow(g2.n, cams2, backward=True, graph=True)
    win.run(*gd2, far, tg2)
    win.run(*gd2, near, tg2, check=False)
    assert not win.check()
    win.run(*gd2, near, tg2)  # resized: the rerun fits
    check_backward(win, plain_views(V, gd2, cams2, near, tg2))
