"""Batched windows whose views have their own Gaussian sets
(VCGS_BATCH_PER_VIEW): each view's images equal a plain render of its own set
bit for bit, its gradients go to its own columns and match the plain backward,
and the view-dependent decode (eqs. (8)-(9)) runs inside a BA window: decode
per keyframe, one batched pass, decode backward per keyframe, pose gradient
through render and decode."""
import numpy as np
import pytest
import torch

from paper_2403_11247_amd import scenes
from tests.gpu_common import FIELDS, dev, gauss_dev, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    vcgs.lib()
    return vcgs


def _targets(cams, seed):
    rng = np.random.default_rng(seed)
    return [(dev(rng.uniform(0, 1, (3, c.height, c.width))), dev(rng.uniform(1.5, 4.5, (c.height, c.width))))
            for c in cams]


def _stack(sets):
    """Per-view attribute sets stacked (V, ., n), as VCGS_BATCH_PER_VIEW reads them."""
    return [torch.stack([s[i] for s in sets]).contiguous() for i in range(5)]


def _plain(V, gd, cam, pose, tg):
    C, D, A, st = V.render_forward(*gd, cam, pose)
    loss, dlc, dld = V.l1_loss(C, D, tg[0], tg[1], 0.5)
    grads, dpose = V.render_backward(st, *gd, cam, pose, dlc, dld, None)
    st.free()
    return (C, D, A), grads, dpose


@pytest.mark.parametrize("graph", [False, True])
def test_own_sets_match_plain_renders(V, graph):
    g = scenes.random_scene(2500, seed=41, xy=1.2)
    base = gauss_dev(g)
    cams = [scenes.Camera(w, h, 0.8 * w, 0.8 * w, w / 2.0, h / 2.0) for (w, h) in [(96, 64), (64, 48), (120, 90)]]
    poses = [scenes.perturb_pose(scenes.identity_pose(), 50 + i, trans=0.1, rot_deg=4.0) for i in range(3)]
    rng = np.random.default_rng(7)
    sets = []
    for v in range(3):  # each view sees different colours, opacities and a slightly moved map
        m, s, q, o, c = [t.clone() for t in base]
        m += dev(rng.normal(0, 0.01, tuple(m.shape)))
        o.mul_(dev(rng.uniform(0.6, 1.0, tuple(o.shape))))
        c.copy_(dev(rng.uniform(0, 1, tuple(c.shape))))
        sets.append((m, s, q, o, c))
    tg = _targets(cams, 9)
    win = V.BatchWindow(g.n, cams, backward=True, graph=graph, per_view=True)
    for _ in range(2):
        win.run(*_stack(sets), poses, tg)
    torch.cuda.synchronize()
    for v in range(3):
        imgs, grads, dpose = _plain(V, sets[v], cams[v], poses[v], tg[v])
        for a, b in zip(win.outs[v], imgs):
            assert torch.equal(a, b), v
        for k in FIELDS:
            got = win.grads[k][v]
            assert rel_err(got.cpu().numpy(), grads[k].cpu().numpy()) <= 1e-5, (v, k)
        assert rel_err(win.dpose[v].cpu().numpy(), dpose.cpu().numpy()) <= 1e-5, v
    say("per-view sets: images bit-exact, gradients per view")


def test_view_dependent_decode_in_a_ba_window(V):
    a = scenes.room_anchors(3000, k=10, seed=6)
    m = scenes.room_mlp_view(seed=6)
    A = [dev(x) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    cams, poses = scenes.ba_window(4, sizes=[(160, 120), (120, 90)])
    tg = _targets(cams, 11)
    centres = [V.camera_centre(p) for p in poses]
    decoded = [V.decode_anchors(*A, cam_centre=c) for c in centres]
    sets = [tuple(d[f] for f in FIELDS) for d in decoded]
    n = int(sets[0][3].shape[0])
    # decode straight into each keyframe's block of the stacked set: the same bits
    stacked = [torch.empty((4,) + tuple(t.shape), device=t.device) for t in sets[0]]
    for v, c in enumerate(centres):
        V.decode_anchors(*A, cam_centre=c, out={f: stacked[i][v] for i, f in enumerate(FIELDS)})
    for x, y in zip(stacked, _stack(sets)):
        assert torch.equal(x, y)
    win = V.BatchWindow(n, cams, backward=True, graph=True, per_view=True)
    win.run(*stacked, poses, tg)
    torch.cuda.synchronize()
    for v in range(4):
        imgs, grads, dpose = _plain(V, sets[v], cams[v], poses[v], tg[v])
        for x, y in zip(win.outs[v], imgs):
            assert torch.equal(x, y), v
        wg = {k: win.grads[k][v] for k in FIELDS}
        ag_win = V.decode_anchors_backward(*A, wg, cam_centre=centres[v])
        ag_ref = V.decode_anchors_backward(*A, grads, cam_centre=centres[v])
        torch.cuda.synchronize()
        for k in ("feat", "W1", "W2", "offset", "cam"):
            assert rel_err(ag_win[k].cpu().numpy(), ag_ref[k].cpu().numpy()) <= 1e-4, (v, k)
        p_win = win.dpose[v].cpu().numpy() + V.pose_grad_from_centre(poses[v], ag_win["cam"]).cpu().numpy()
        p_ref = dpose.cpu().numpy() + V.pose_grad_from_centre(poses[v], ag_ref["cam"]).cpu().numpy()
        assert rel_err(p_win, p_ref) <= 1e-4, v
    say(f"view-dependent decode in a {len(cams)}-keyframe window: {n} Gaussians per view")


def test_per_view_graph_replays_follow_new_poses_and_sets(V):
    """The captured per-view pass replayed with new poses and new per-view
    sets each time (plain renders between the replays): every replay's images
    equal the plain renders bit for bit and its gradients match."""
    g = scenes.random_scene(2000, seed=43, xy=1.2)
    base = gauss_dev(g)
    cams = [scenes.Camera(w, h, 0.8 * w, 0.8 * w, w / 2.0, h / 2.0) for (w, h) in [(96, 64), (120, 90)]]
    tg = _targets(cams, 12)
    win = V.BatchWindow(g.n, cams, backward=True, graph=True, per_view=True)
    rng = np.random.default_rng(13)
    for it in range(3):
        poses = [scenes.perturb_pose(scenes.identity_pose(), 70 + 3 * it + v, trans=0.1, rot_deg=4.0)
                 for v in range(2)]
        sets = []
        for v in range(2):
            m, s, q, o, c = [t.clone() for t in base]
            m += dev(rng.normal(0, 0.02, tuple(m.shape)))
            c.copy_(dev(rng.uniform(0, 1, tuple(c.shape))))
            sets.append((m, s, q, o, c))
        win.run(*_stack(sets), poses, tg)
        torch.cuda.synchronize()
        for v in range(2):
            imgs, grads, dpose = _plain(V, sets[v], cams[v], poses[v], tg[v])
            for a_, b_ in zip(win.outs[v], imgs):
                assert torch.equal(a_, b_), (it, v)
            for k in FIELDS:
                assert rel_err(win.grads[k][v].cpu().numpy(), grads[k].cpu().numpy()) <= 1e-5, (it, v, k)
            assert rel_err(win.dpose[v].cpu().numpy(), dpose.cpu().numpy()) <= 1e-5, (it, v)
    say("per-view graph: 3 replays with new poses and sets match plain renders")
