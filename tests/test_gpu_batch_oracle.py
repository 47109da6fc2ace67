"""The batched window (local bundle adjustment, Sec. 3.5) and the autograd
Functions against the oracle.

* BatchRender (vcgs_render_batch_forward / _backward, the loss outside the
  library): every view's images against the oracle (unflagged pixels within
  1e-4, flagged pixels equal to one of the oracle's enumerated outcomes), the
  Gaussian gradients summed over the views and each view's SE(3) pose gradient
  against the sum of the oracle's per-view adjoints, element by element --
  for each compositing-backward launch shape (1, 2, 4 pixels per lane) and
  as a replayed hipGraph.
* A BA step whose per-view upstream gradient is L1 colour + 0.5 L1 depth +
  0.2 (1 - SSIM): the loss kernels against the oracle's losses on the same
  images, the backward against the oracle's adjoint.
* RenderFn, BatchRenderFn and DecodeFn: gradients of a scalar loss through
  torch.autograd against the direct calls and the oracle.
"""
import numpy as np
import pytest
import torch

from oracle import decode as odec, raster, track as otrack
from paper_2403_11247_amd import scenes
from tests.gpu_common import FIELDS, GRAD_REL_TOL, compare_images, dev, gauss_dev, grad_check, rel_err, say, zero_at

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


def view_refs(g, cams, poses, outs):
    """Per view: the oracle's render, the comparison (variant map) and the
    mask of pixels that get no upstream gradient (an ambiguous outcome, or
    the 0.99 clamp within FP32 noise)."""
    refs = []
    for i, (c, p) in enumerate(zip(cams, poses)):
        ref = raster.render(g, c, p)
        r = compare_images(*outs[i], ref, g=g, cam=c)
        assert r["pass_"], (i, r)
        skip = (r["variant"] < 0) | ((ref["flags"] & 4) != 0)
        refs.append(dict(ref=ref, variant=np.maximum(r["variant"], 0), skip=skip, flagged=r["flagged"]))
    return refs


def oracle_window_grads(g, cams, poses, refs, ups):
    tot = {k: 0.0 for k in FIELDS}
    dpose = []
    for c, p, rf, up in zip(cams, poses, refs, ups):
        gr = raster.render_backward(g, c, p, rf["ref"], *up, variant=rf["variant"])
        for k in FIELDS:
            tot[k] = tot[k] + gr[k]
        dpose.append(gr["pose"])
    return tot, np.stack(dpose)


def check_window(grads, dpose, tot, dpose_ref, what):
    errs = {k: grad_check(f"{what} {k}", grads[k].cpu().numpy(), tot[k]) for k in FIELDS}
    for i in range(dpose_ref.shape[0]):
        errs[f"pose{i}"] = grad_check(f"{what} pose {i}", dpose[i].cpu().numpy(), dpose_ref[i])
    say(what, {k: "%.1e" % v for k, v in errs.items()})


@pytest.mark.parametrize("ppl,graph", [(1, False), (2, False), (4, False), (1, True)])
def test_batch_gradients_match_oracle(V, ppl, graph):
    saved = V.get_option("ppl_bwd")
    V.set_option("ppl_bwd", ppl)
    try:
        g = scenes.random_scene(3000, seed=4, xy=1.2)
        gd = gauss_dev(g)
        cams, poses = small_window(seed=10)
        br = V.BatchRender(g.n, cams, graph=graph)
        outs = br.forward(*gd, poses)
        torch.cuda.synchronize()
        refs = view_refs(g, cams, poses, outs)
        ups = [zero_at(scenes.upstream_grads(c.width, c.height, seed=40 + i), rf["skip"])
               for i, (c, rf) in enumerate(zip(cams, refs))]
        grads, dpose = br.backward(*[[dev(u[j]) for u in ups] for j in range(3)])
        torch.cuda.synchronize()
        say(f"window ppl {ppl} graph {graph}: pairs {br.pairs}, flagged {[rf['flagged'] for rf in refs]}")
        tot, dpose_ref = oracle_window_grads(g, cams, poses, refs, ups)
        check_window(grads, dpose, tot, dpose_ref, f"window ppl {ppl}")
    finally:
        V.set_option("ppl_bwd", saved)


def test_batch_graph_replays_new_poses_match_oracle(V):
    """The captured forward and backward graphs replayed at new poses."""
    g = scenes.random_scene(2500, seed=6, xy=1.2)
    gd = gauss_dev(g)
    cams, _ = small_window(4, seed=50)
    br = V.BatchRender(g.n, cams, graph=True)
    for it in range(3):
        _, poses = small_window(4, seed=60 + 7 * it)
        outs = br.forward(*gd, poses)
        torch.cuda.synchronize()
        refs = view_refs(g, cams, poses, outs)
        ups = [zero_at(scenes.upstream_grads(c.width, c.height, seed=70 + i + it), rf["skip"])
               for i, (c, rf) in enumerate(zip(cams, refs))]
        grads, dpose = br.backward(*[[dev(u[j]) for u in ups] for j in range(3)])
        torch.cuda.synchronize()
        tot, dpose_ref = oracle_window_grads(g, cams, poses, refs, ups)
        check_window(grads, dpose, tot, dpose_ref, f"graph replay {it}")


def _l1_ssim_upstream_oracle(C, D, tC, tD, w_depth=0.5, w_ssim=0.2):
    """The BA loss's upstream gradient and value computed by the oracle on the
    GPU's images: mean L1 colour + w_depth mean L1 depth + w_ssim (1 - SSIM)."""
    C, D = C.astype(np.float64), D.astype(np.float64)
    npix = D.size
    l_s, g_s, _ = otrack.ssim(C, tC)
    dlc = np.sign(C - tC) / npix + w_ssim * g_s
    dld = w_depth * np.sign(D - tD) / npix
    loss = (np.abs(C - tC).sum() + w_depth * np.abs(D - tD).sum()) / npix
    return loss, w_ssim * l_s, dlc, dld


def test_ba_step_l1_ssim_matches_oracle(V):
    g = scenes.random_scene(3000, seed=8, xy=1.2)
    gd = gauss_dev(g)
    cams, poses = small_window(seed=20)
    targets = [raster.render(g, c, scenes.perturb_pose(p, 200 + i, trans=0.02, rot_deg=1.0))
               for i, (c, p) in enumerate(zip(cams, poses))]
    br = V.BatchRender(g.n, cams)
    outs = br.forward(*gd, poses)
    torch.cuda.synchronize()
    refs = view_refs(g, cams, poses, outs)
    ups = []
    for i, (c, rf, t) in enumerate(zip(cams, refs, targets)):
        tC, tD = t["color"].astype(np.float32), t["depth"].astype(np.float32)
        C, D, _ = outs[i]
        l1, dlc, dld = V.l1_loss(C, D, dev(tC), dev(tD), 0.5)
        ls, dlc = V.ssim_loss(C, dev(tC), weight=0.2, dl_dcolor=dlc)
        torch.cuda.synchronize()
        ol1, ols, odlc, odld = _l1_ssim_upstream_oracle(C.cpu().numpy(), D.cpu().numpy(), tC, tD)
        assert abs(float(l1[0]) - ol1) <= 1e-5 * ol1, (i, float(l1[0]), ol1)
        assert abs(float(ls[0]) - ols) <= 1e-4 * abs(ols) + 1e-7, (i, float(ls[0]), ols)
        gdlc, gdld = dlc.cpu().numpy(), dld.cpu().numpy()
        assert np.array_equal(np.sign(gdld), np.sign(odld)), i
        np.testing.assert_allclose(gdld, odld, rtol=1e-6, atol=0)
        np.testing.assert_allclose(gdlc, odlc, rtol=1e-3, atol=1e-4 * np.abs(odlc).max())
        ups.append(zero_at((gdlc, gdld, np.zeros_like(gdld)), rf["skip"]))
    grads, dpose = br.backward([dev(u[0]) for u in ups], [dev(u[1]) for u in ups], None)
    torch.cuda.synchronize()
    tot, dpose_ref = oracle_window_grads(g, cams, poses, refs, ups)
    check_window(grads, dpose, tot, dpose_ref, "BA step L1+SSIM")


def test_full_size_view_pose_gradient_in_a_window(V):
    """A 1200x680 room view and two small views in one batched pass: the
    full-size view's pose gradient and the window's Gaussian gradients against
    the oracle."""
    a = scenes.room_anchors(8000, k=10, seed=3)
    m = scenes.room_mlp(seed=3)
    dec = odec.decode(a, m)
    g = scenes.Gaussians(*[dec[f].astype(np.float32) for f in FIELDS])
    gd = gauss_dev(g)
    cam, pose = scenes.room_camera()
    small = scenes.Camera(320, 240, 160.0, 160.0, 160.0, 120.0)
    cams = [small, cam, small]
    poses = [scenes.perturb_pose(pose, 300, trans=0.2, rot_deg=5.0), pose,
             scenes.perturb_pose(pose, 301, trans=0.3, rot_deg=8.0)]
    br = V.BatchRender(g.n, cams)
    outs = br.forward(*gd, poses)
    torch.cuda.synchronize()
    refs = view_refs(g, cams, poses, outs)
    ups = [zero_at(scenes.upstream_grads(c.width, c.height, seed=80 + i), rf["skip"])
           for i, (c, rf) in enumerate(zip(cams, refs))]
    grads, dpose = br.backward(*[[dev(u[j]) for u in ups] for j in range(3)])
    torch.cuda.synchronize()
    say("full-size window: flagged", [rf["flagged"] for rf in refs], "pairs", br.pairs)
    tot, dpose_ref = oracle_window_grads(g, cams, poses, refs, ups)
    check_window(grads, dpose, tot, dpose_ref, "full-size window")


def test_stale_batch_backward_is_refused(V):
    g = scenes.random_scene(500, seed=1)
    gd = gauss_dev(g)
    cams, poses = small_window(2, seed=3)
    a = V.BatchRender(g.n, cams)
    b = V.BatchRender(g.n, cams[:1])
    a.forward(*gd, poses)
    b.forward(*gd, poses[:1])
    with pytest.raises(V.VcgsError):
        a.backward()


def _weights(cam, seed, skip=None):
    up = scenes.upstream_grads(cam.width, cam.height, seed=seed)
    return up if skip is None else zero_at(up, skip)


def test_render_fn_autograd_matches_direct_and_oracle(V):
    g = scenes.random_scene(2000, seed=11, xy=1.2)
    cam = scenes.random_camera()
    pose = scenes.perturb_pose(scenes.identity_pose(), 5, trans=0.05, rot_deg=2.0)
    ref = raster.render(g, cam, pose)
    gd = gauss_dev(g)
    C0, D0, A0, st = V.render_forward(*gd, cam, pose)
    r = compare_images(C0, D0, A0, ref, g=g, cam=cam, pix_state=st.pixel_state(cam.width, cam.height))
    assert r["pass_"], r
    up = _weights(cam, 12, (r["variant"] < 0) | ((ref["flags"] & 4) != 0))
    w = [dev(u) for u in up]
    leaves = [t.clone().requires_grad_(True) for t in gd]
    tangent = torch.zeros(6, device="cuda", requires_grad=True)
    C, D, A = V.render(*leaves, cam, pose, pose_tangent=tangent)
    loss = (C * w[0]).sum() + (D * w[1]).sum() + (A * w[2]).sum()
    got = torch.autograd.grad(loss, leaves + [tangent], retain_graph=True)
    again = torch.autograd.grad(loss, leaves + [tangent])  # the retained graph replays
    direct, dpose = V.render_backward(st, *gd, cam, pose, *w)
    torch.cuda.synchronize()
    gref = raster.render_backward(g, cam, pose, ref, *up, variant=np.maximum(r["variant"], 0))
    for k, a, b in zip(FIELDS + ("pose",), got, again):
        d = direct[k] if k != "pose" else dpose
        assert rel_err(a.cpu().numpy(), d.cpu().numpy()) <= 1e-6, k
        assert rel_err(b.cpu().numpy(), d.cpu().numpy()) <= 1e-6, k
        grad_check(f"RenderFn {k}", a.cpu().numpy(), gref[k])
    st.free()


def test_render_views_autograd_matches_direct(V):
    g = scenes.random_scene(2500, seed=13, xy=1.2)
    gd = gauss_dev(g)
    cams, poses = small_window(3, seed=90)
    br = V.BatchRender(g.n, cams)
    leaves = [t.clone().requires_grad_(True) for t in gd]
    tangents = torch.zeros((3, 6), device="cuda", requires_grad=True)
    imgs = V.render_views(*leaves, br, poses, pose_tangents=tangents)
    ws = [[dev(u) for u in _weights(c, 20 + i)] for i, c in enumerate(cams)]
    loss = sum((C * w[0]).sum() + (D * w[1]).sum() + (A * w[2]).sum() for (C, D, A), w in zip(imgs, ws))
    got = torch.autograd.grad(loss, leaves + [tangents])
    # the same window as per-view RenderFn calls
    tot = {k: 0.0 for k in FIELDS}
    dps = []
    for c, p, w in zip(cams, poses, ws):
        C, D, A, st = V.render_forward(*gd, c, p)
        gr, dp = V.render_backward(st, *gd, c, p, *w)
        for k in FIELDS:
            tot[k] = tot[k] + gr[k]
        dps.append(dp)
        st.free()
    torch.cuda.synchronize()
    for k, a in zip(FIELDS, got):
        assert rel_err(a.cpu().numpy(), tot[k].cpu().numpy()) <= 1e-5, k
    assert rel_err(got[-1].cpu().numpy(), torch.stack(dps).cpu().numpy()) <= 1e-5


def test_decode_fn_autograd_matches_direct_and_oracle(V):
    a = scenes.room_anchors(600, k=10, seed=21)
    m = scenes.room_mlp(k=10, seed=5)
    n = a.n * a.k
    rng = np.random.default_rng(3)
    dG = {"mean": rng.normal(size=(3, n)), "scale": rng.normal(size=(3, n)) * 10, "quat": rng.normal(size=(4, n)),
          "opacity": rng.normal(size=n), "color": rng.normal(size=(3, n))}
    dG = {k: v.astype(np.float32) for k, v in dG.items()}
    names = ("xa", "feat", "scaling", "offset", "W1", "b1", "W2", "b2")
    vals = [a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2]
    leaves = [dev(v).requires_grad_(True) for v in vals]
    outs = V.decode(*leaves)
    loss = sum((o * dev(dG[k])).sum() for o, k in zip(outs, FIELDS))
    got = dict(zip(names, torch.autograd.grad(loss, leaves)))
    direct = V.decode_anchors_backward(*[dev(v) for v in vals], {k: dev(v) for k, v in dG.items()})
    fwd = odec.decode(a, m)
    ref = odec.decode_backward(a, m, fwd, dG)
    torch.cuda.synchronize()
    for k in names:
        assert rel_err(got[k].cpu().numpy(), direct[k].cpu().numpy()) <= 1e-6, k
        e = rel_err(got[k].cpu().numpy().reshape(np.shape(ref[k])), ref[k])
        assert e <= 1e-4, (k, e)


@pytest.mark.parametrize("graph", [False, True])
def test_repeated_batch_backward_after_one_forward(V, graph):
    """Two backwards of one batched forward give the same gradients (the
    gradient slots start from zero again), also when the backward is a
    replayed graph; a later forward and backward agree with the first pass."""
    g = scenes.random_scene(2000, seed=15, xy=1.2)
    gd = gauss_dev(g)
    cams, poses = small_window(3, seed=95)
    br = V.BatchRender(g.n, cams, graph=graph)
    ups = [[dev(u) for u in scenes.upstream_grads(c.width, c.height, seed=30 + i)] for i, c in enumerate(cams)]
    first = None
    for it in range(2):
        br.forward(*gd, poses)
        for rep in range(2):
            grads, dpose = br.backward([u[0] for u in ups], [u[1] for u in ups], [u[2] for u in ups])
            torch.cuda.synchronize()
            got = {k: grads[k].cpu().numpy().copy() for k in FIELDS}
            got["pose"] = dpose.cpu().numpy().copy()
            if first is None:
                first = got
            for k in got:
                assert rel_err(got[k], first[k]) <= 1e-6, (it, rep, k)
