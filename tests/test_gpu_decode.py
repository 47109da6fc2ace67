"""GPU parity of the anchor decode (FP32 MFMA) and its adjoint against the
numpy FP64 oracle, with and without the residual codebook and the mask."""
import numpy as np
import pytest
import torch

from oracle import decode as odec
from paper_2403_11247_amd import scenes
from tests.gpu_common import FIELDS, dev, rel_err, say

pytestmark = pytest.mark.gpu

DEC_TOL = 1e-5      # decoded attributes, relative to the attribute's scale
DEC_GRAD_TOL = 1e-4  # per-tensor relative L2 of decode gradients


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    vcgs.lib()
    return vcgs


def run_decode(V, a, m, books=None, idx=None, mask=None, eps=0.01):
    from paper_2403_11247_amd.vcgs import decode_anchors
    return decode_anchors(dev(a.xa), dev(a.feat), dev(a.scaling), dev(a.offset), dev(m.W1), dev(m.b1), dev(m.W2),
                          dev(m.b2), None if books is None else dev(books),
                          None if idx is None else dev(idx, torch.int32), None if mask is None else dev(mask), eps)


def check_decode(out, ref):
    for f in FIELDS:
        a = out[f].cpu().numpy().astype(np.float64)
        b = ref[f]
        scale_ = max(np.abs(b).max(), 1e-30)
        err = np.abs(a - b).max() / scale_
        say("decode", f, "max err / max |ref| = %.2e" % err)
        assert err <= DEC_TOL, (f, err)


@pytest.mark.parametrize("na,k", [(2000, 10), (37, 10), (513, 3), (100, 16), (16, 1)])
def test_decode_forward(V, na, k):
    a = scenes.room_anchors(na, k=k, seed=na)
    m = scenes.room_mlp(k=k, seed=1)
    say("decode forward na", na, "k", k)
    out = run_decode(V, a, m)
    torch.cuda.synchronize()
    check_decode(out, odec.decode(a, m))


def test_decode_codebook_and_mask(V):
    a = scenes.room_anchors(1500, k=10, seed=3)
    m = scenes.room_mlp(k=10, seed=2)
    n = a.n * a.k
    logits, books, idx = scenes.mask_and_codebook(n, size=4096, mask_mu=0.0, mask_sigma=3.0)
    # keep logits away from the threshold so FP32 and FP64 agree on every keep decision
    thr = np.log(0.01 / 0.99)
    logits[np.abs(logits - thr) < 1e-4] += 1e-3
    out = run_decode(V, a, m, books, idx, logits)
    torch.cuda.synchronize()
    ref = odec.decode(a, m, books, idx, logits)
    check_decode(out, ref)
    assert np.array_equal(out["opacity"].cpu().numpy() == 0, ref["opacity"] == 0)


def check_decode_backward(V, a, m, books=None, idx=None, mask=None, seed=0):
    from paper_2403_11247_amd.vcgs import decode_anchors_backward
    n = a.n * a.k
    rng = np.random.default_rng(seed)
    dG = {"mean": rng.normal(size=(3, n)), "scale": rng.normal(size=(3, n)) * 10, "quat": rng.normal(size=(4, n)),
          "opacity": rng.normal(size=n), "color": rng.normal(size=(3, n))}
    dG = {k: v.astype(np.float32) for k, v in dG.items()}
    fwd = odec.decode(a, m, books, idx, mask)
    ref = odec.decode_backward(a, m, fwd, dG, books, idx, mask)
    got = decode_anchors_backward(dev(a.xa), dev(a.feat), dev(a.scaling), dev(a.offset), dev(m.W1), dev(m.b1),
                                  dev(m.W2), dev(m.b2), {k: dev(v) for k, v in dG.items()},
                                  None if books is None else dev(books),
                                  None if idx is None else dev(idx, torch.int32),
                                  None if mask is None else dev(mask), 0.01)
    torch.cuda.synchronize()
    keys = ["feat", "W1", "b1", "W2", "b2", "offset", "scaling", "xa"]
    if books is not None:
        keys.append("books")
        ref["books"] = np.stack(ref["books"])
    if mask is not None:
        keys.append("mask_logit")
    for k in keys:
        e = rel_err(got[k].cpu().numpy().reshape(np.shape(ref[k])), ref[k])
        say("decode backward", k, "rel err %.2e" % e)
        assert e <= DEC_GRAD_TOL, (k, e)


@pytest.mark.parametrize("na,k", [(2000, 10), (45, 7), (300, 16)])
def test_decode_backward(V, na, k):
    a = scenes.room_anchors(na, k=k, seed=na + 1)
    m = scenes.room_mlp(k=k, seed=3)
    check_decode_backward(V, a, m)


def test_decode_backward_codebook_and_mask(V):
    a = scenes.room_anchors(800, k=10, seed=9)
    m = scenes.room_mlp(k=10, seed=4)
    n = a.n * a.k
    logits, books, idx = scenes.mask_and_codebook(n, size=256, mask_mu=0.0, mask_sigma=3.0)
    thr = np.log(0.01 / 0.99)
    logits[np.abs(logits - thr) < 1e-4] += 1e-3
    check_decode_backward(V, a, m, books, idx, logits)


def test_decode_full_room(V):
    a = scenes.room_anchors(40000, k=10)
    m = scenes.room_mlp()
    say("decode room 40k anchors")
    out = run_decode(V, a, m)
    torch.cuda.synchronize()
    check_decode(out, odec.decode(a, m))


# view-dependent decode: MLP input [f_a, delta, d] from the camera centre (eqs. (8)-(9))

CAM_C = np.array([2.9, 2.4, 1.3], np.float32)


@pytest.mark.parametrize("na,k", [(2000, 10), (37, 10), (300, 16), (16, 1)])
def test_view_decode_forward(V, na, k):
    from paper_2403_11247_amd.vcgs import decode_anchors
    a = scenes.room_anchors(na, k=k, seed=na + 5)
    m = scenes.room_mlp_view(k=k, seed=2, view_gain=4.0)
    say("view decode forward na", na, "k", k)
    out = decode_anchors(dev(a.xa), dev(a.feat), dev(a.scaling), dev(a.offset), dev(m.W1), dev(m.b1), dev(m.W2),
                         dev(m.b2), cam_centre=CAM_C)
    torch.cuda.synchronize()
    check_decode(out, odec.decode(a, m, cam=CAM_C.astype(np.float64)))


@pytest.mark.parametrize("na,k,masked", [(2000, 10, False), (45, 7, False), (800, 10, True)])
def test_view_decode_backward(V, na, k, masked):
    from paper_2403_11247_amd.vcgs import decode_anchors_backward
    a = scenes.room_anchors(na, k=k, seed=na + 7)
    m = scenes.room_mlp_view(k=k, seed=5, view_gain=4.0)
    n = a.n * a.k
    mask = None
    if masked:
        mask, _, _ = scenes.mask_and_codebook(n, size=16, mask_mu=0.0, mask_sigma=3.0)
        thr = np.log(0.01 / 0.99)
        mask[np.abs(mask - thr) < 1e-4] += 1e-3
    rng = np.random.default_rng(3)
    dG = {"mean": rng.normal(size=(3, n)), "scale": rng.normal(size=(3, n)) * 10, "quat": rng.normal(size=(4, n)),
          "opacity": rng.normal(size=n), "color": rng.normal(size=(3, n))}
    dG = {kk: v.astype(np.float32) for kk, v in dG.items()}
    c64 = CAM_C.astype(np.float64)
    fwd = odec.decode(a, m, mask_logit=mask, cam=c64)
    ref = odec.decode_backward(a, m, fwd, dG, mask_logit=mask, cam=c64)
    got = decode_anchors_backward(dev(a.xa), dev(a.feat), dev(a.scaling), dev(a.offset), dev(m.W1), dev(m.b1),
                                  dev(m.W2), dev(m.b2), {kk: dev(v) for kk, v in dG.items()},
                                  mask_logit=None if mask is None else dev(mask), cam_centre=CAM_C)
    torch.cuda.synchronize()
    for kk in ["feat", "W1", "b1", "W2", "b2", "offset", "scaling", "xa", "cam"] + (["mask_logit"] if masked else []):
        e = rel_err(got[kk].cpu().numpy().reshape(np.shape(ref[kk])), ref[kk])
        say("view decode backward", kk, "rel err %.2e" % e)
        assert e <= DEC_GRAD_TOL, (kk, e)


def test_view_decode_pose_gradient_helper(V):
    from paper_2403_11247_amd.vcgs import camera_centre, pose_grad_from_centre
    pose = scenes.look_at((1.0, 2.0, 1.5), (4.0, 3.0, 1.0))
    np.testing.assert_allclose(camera_centre(pose), [1.0, 2.0, 1.5], atol=1e-5)
    d = np.array([0.3, -0.2, 0.9])
    g = pose_grad_from_centre(pose, dev(d)).cpu().numpy()
    np.testing.assert_allclose(g, odec.pose_grad_from_centre(pose.R, d), rtol=1e-5, atol=1e-6)
    # several poses at once, added to what the pose gradients already hold
    rng = np.random.default_rng(4)
    poses = [scenes.perturb_pose(pose, 30 + i, trans=0.3, rot_deg=40.0) for i in range(5)]
    dc = rng.normal(size=(5, 3))
    base = rng.normal(size=(5, 6))
    got = V.add_centre_pose_grad(poses, dev(dc), dev(base).contiguous()).cpu().numpy()
    want = base + np.stack([odec.pose_grad_from_centre(p.R, dc[i]) for i, p in enumerate(poses)])
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-6)


def _centres(V_, seed):
    rng = np.random.default_rng(seed)
    return (CAM_C + rng.uniform(-0.6, 0.6, (V_, 3))).astype(np.float32)


@pytest.mark.parametrize("na,k,nv,extras", [(300, 10, 3, False), (37, 10, 1, False), (45, 7, 16, False),
                                            (200, 10, 4, True)])
def test_decode_views_forward_and_backward(V, na, k, nv, extras):
    """One launch for nv camera centres (a keyframe window): every view's block
    equals the single-centre decode bit for bit and matches the oracle; the
    backward's anchor, MLP, codebook and mask gradients match the oracle's sums
    over the views, and its centre gradients match the oracle per view."""
    a = scenes.room_anchors(na, k=k, seed=na + 11)
    m = scenes.room_mlp_view(k=k, seed=7, view_gain=4.0)
    n = a.n * a.k
    books = idx = mask = None
    if extras:
        mask, books, idx = scenes.mask_and_codebook(n, size=64, mask_mu=0.0, mask_sigma=3.0)
        thr = np.log(0.01 / 0.99)
        mask[np.abs(mask - thr) < 1e-4] += 1e-3
    cs = _centres(nv, na)
    A = [dev(x) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    kw = dict(books=None if books is None else dev(books), idx=None if idx is None else dev(idx, torch.int32),
              mask_logit=None if mask is None else dev(mask))
    say("decode views na", na, "k", k, "views", nv, "codebook+mask", extras)
    got = V.decode_anchors_views(*A, cs, **kw)
    rng = np.random.default_rng(na)
    dG = {"mean": rng.normal(size=(nv, 3, n)), "scale": rng.normal(size=(nv, 3, n)) * 10,
          "quat": rng.normal(size=(nv, 4, n)), "opacity": rng.normal(size=(nv, n)),
          "color": rng.normal(size=(nv, 3, n))}
    dG = {kk: v.astype(np.float32) for kk, v in dG.items()}
    gb = V.decode_anchors_views_backward(*A, {kk: dev(v) for kk, v in dG.items()}, cs, **kw)
    torch.cuda.synchronize()
    keys = ["feat", "W1", "b1", "W2", "b2", "offset", "scaling", "xa"] + (["books", "mask_logit"] if extras else [])
    sums = None
    for v in range(nv):
        one = V.decode_anchors(*A, cam_centre=cs[v], **kw)
        torch.cuda.synchronize()
        for f in FIELDS:
            assert torch.equal(got[f][v], one[f]), (v, f)
        c64 = cs[v].astype(np.float64)
        fwd = odec.decode(a, m, books, idx, mask, cam=c64)
        check_decode({f: got[f][v] for f in FIELDS}, fwd)
        ref = odec.decode_backward(a, m, fwd, {kk: x[v] for kk, x in dG.items()}, books, idx, mask, cam=c64)
        if extras:
            ref["books"] = np.stack(ref["books"])
        e = rel_err(gb["cam"][v].cpu().numpy(), ref["cam"])
        assert e <= DEC_GRAD_TOL, ("cam", v, e)
        sums = {kk: np.asarray(ref[kk], np.float64) for kk in keys} if sums is None else \
            {kk: sums[kk] + np.asarray(ref[kk], np.float64) for kk in keys}
    for kk in keys:
        e = rel_err(gb[kk].cpu().numpy().reshape(np.shape(sums[kk])), sums[kk])
        say("decode views backward", kk, "rel err %.2e" % e)
        assert e <= DEC_GRAD_TOL, (kk, e)


def test_decode_views_limits(V):
    a = scenes.room_anchors(40, k=10, seed=2)
    m = scenes.room_mlp_view(k=10, seed=2)
    A = [dev(x) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    with pytest.raises(V.VcgsError):
        V.decode_anchors_views(*A, _centres(17, 1))
    with pytest.raises(V.VcgsError):
        V.decode_anchors_views(*A, np.zeros((0, 3), np.float32))


def test_decode_with_no_anchors(V):
    """An empty anchor set decodes to empty sets, and every backward form
    returns zero weight and camera-centre gradients (not uninitialised memory)."""
    m = scenes.room_mlp(seed=1)
    mv = scenes.room_mlp_view(seed=1)
    empty = [torch.zeros((3, 0), device="cuda"), torch.zeros((0, 32), device="cuda"),
             torch.zeros((3, 0), device="cuda"), torch.zeros((0, 10, 3), device="cuda")]
    for mm, kw in ((m, {}), (mv, {"cam_centre": CAM_C})):
        A = empty + [dev(x) for x in (mm.W1, mm.b1, mm.W2, mm.b2)]
        G = V.decode_anchors(*A, **kw)
        assert all(G[f].numel() == 0 for f in FIELDS)
        ag = V.decode_anchors_backward(*A, G, **kw)
        torch.cuda.synchronize()
        for k in ("W1", "b1", "W2", "b2") + (("cam",) if kw else ()):
            assert bool((ag[k] == 0).all()), k
    A = empty + [dev(x) for x in (mv.W1, mv.b1, mv.W2, mv.b2)]
    cs = _centres(3, 5)
    Gs = V.decode_anchors_views(*A, cs)
    ag = V.decode_anchors_views_backward(*A, Gs, cs)
    torch.cuda.synchronize()
    for k in ("W1", "b1", "W2", "b2", "cam"):
        assert bool((ag[k] == 0).all()), k


def test_decode_views_full_window_size(V):
    """The BA window's map size (50k anchors x 10) at three camera centres in
    one launch: every view's 500k decoded Gaussians against the oracle."""
    a = scenes.room_anchors(50000, k=10, spacing=0.05, seed=1)
    m = scenes.room_mlp_view(seed=1)
    A = [dev(x) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    _, poses = scenes.ba_window(3)
    cs = np.stack([V.camera_centre(p) for p in poses]).astype(np.float32)
    got = V.decode_anchors_views(*A, cs)
    torch.cuda.synchronize()
    for v in range(3):
        check_decode({f: got[f][v] for f in FIELDS}, odec.decode(a, m, cam=cs[v].astype(np.float64)))


def test_decode_full_room_codebook_and_mask(V):
    """The compacted room's decode at full size (40k anchors x 10, mask logits
    N(2, 1), 2 x 4096 x 7 codebooks) against the oracle."""
    a = scenes.room_anchors(40000, k=10)
    m = scenes.room_mlp(seed=0)
    n = a.n * a.k
    logits, books, idx = scenes.mask_and_codebook(n)
    thr = np.log(0.01 / 0.99)
    logits[np.abs(logits - thr) < 1e-4] += 1e-3
    out = run_decode(V, a, m, books, idx, logits)
    torch.cuda.synchronize()
    ref = odec.decode(a, m, books, idx, logits)
    check_decode(out, ref)
    assert np.array_equal(out["opacity"].cpu().numpy() == 0, ref["opacity"] == 0)


def test_decode_backward_full_room_codebook_and_mask(V):
    """The compacted room's decode adjoint at full size: the codebook rows'
    straight-through sums come from ~100 per-block LDS tables, checked with
    every other gradient against the oracle."""
    a = scenes.room_anchors(40000, k=10, seed=4)
    m = scenes.room_mlp(seed=4)
    n = a.n * a.k
    logits, books, idx = scenes.mask_and_codebook(n, mask_mu=0.0, mask_sigma=3.0)
    thr = np.log(0.01 / 0.99)
    logits[np.abs(logits - thr) < 1e-4] += 1e-3
    check_decode_backward(V, a, m, books, idx, logits, seed=9)
