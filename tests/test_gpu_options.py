"""Every launch configuration the autotuner may pick (pixels per lane of the
forward and backward compositing, culling, block order) gives the same
images bit for bit, the same gradients up to summation order (1e-5
relative), and gradients within the oracle's bars (1e-3 relative per tensor
and element by element), on a ragged image whose tiles have long lists; the
stage-timing mask times only the selected stages."""
import numpy as np
import pytest
import torch

from oracle import raster
from paper_2403_11247_amd import autotune, scenes
from tests.gpu_common import FIELDS, compare_images, dev, gauss_dev, grad_check, rel_err, say, zero_at

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    vcgs.lib()
    return vcgs


def run(V, gd, cam, pose, up, pix=False):
    C, D, A, st = V.render_forward(*gd, cam, pose)
    ps = st.pixel_state(cam.width, cam.height) if pix else None
    grads, dpose = V.render_backward(st, *gd, cam, pose, *up)
    st.free()
    torch.cuda.synchronize()
    return (C, D, A, grads, dpose, ps) if pix else (C, D, A, grads, dpose)


def test_all_launch_configurations_agree(V):
    g = scenes.random_scene(6000, seed=11, xy=1.3, log_scale=(0.02, 0.12))
    gd = gauss_dev(g)
    cam = scenes.Camera(200, 136, 160.0, 160.0, 100.0, 68.0)
    pose = scenes.perturb_pose(scenes.identity_pose(), 5, trans=0.05, rot_deg=2.0)
    up_h = scenes.upstream_grads(cam.width, cam.height, seed=4)
    ref = raster.render(g, cam, pose)
    saved = autotune.current()
    try:
        autotune.apply({"ppl_fwd": 1, "ppl_bwd": 1, "cull": 1, "sched": 0})
        # the forward fixes which outcome each flagged pixel takes; the oracle follows it
        C0, D0, A0, _, _, ps = run(V, gd, cam, pose, [dev(x) for x in up_h], pix=True)
        r = compare_images(C0, D0, A0, ref, g=g, cam=cam, pix_state=ps)
        assert r["pass_"], r
        up_h = zero_at(up_h, (r["variant"] < 0) | ((ref["flags"] & 4) != 0))
        up = [dev(x) for x in up_h]
        gref = raster.render_backward(g, cam, pose, ref, *up_h, variant=np.maximum(r["variant"], 0))
        _, _, _, G0, P0 = run(V, gd, cam, pose, up)
        n = 0
        for cfg in autotune.candidates(True):
            autotune.apply(cfg)
            C, D, A, G, P = run(V, gd, cam, pose, up)
            assert torch.equal(C, C0) and torch.equal(D, D0) and torch.equal(A, A0), cfg
            worst = max(rel_err(G[k].cpu().numpy(), G0[k].cpu().numpy()) for k in FIELDS)
            worst = max(worst, rel_err(P.cpu().numpy(), P0.cpu().numpy()))
            assert worst <= 1e-5, (cfg, worst)
            for k in FIELDS:
                grad_check(f"{cfg} {k}", G[k].cpu().numpy(), gref[k])
            grad_check(f"{cfg} pose", P.cpu().numpy(), gref["pose"])
            n += 1
        say("launch configurations checked against the oracle:", n)
    finally:
        autotune.apply(saved)


def test_stage_timing_mask(V):
    """vcgs_profile_stages: with one stage selected only that stage records
    launches; the default times every stage of a forward + backward."""
    g = scenes.random_scene(3000, seed=5)
    gd = gauss_dev(g)
    cam = scenes.Camera(128, 96, 100.0, 100.0, 64.0, 48.0)
    pose = scenes.identity_pose()
    up = [dev(x) for x in scenes.upstream_grads(cam.width, cam.height, seed=2)]

    def step():
        _, _, _, st = V.render_forward(*gd, cam, pose)
        V.render_backward(st, *gd, cam, pose, *up)
        st.free()

    try:
        V.profile_stages(["composite_bwd"])
        V.profile_enable(True)
        step()
        step()
        prof = V.profile_read()
        assert prof["composite_bwd"][1] == 2 and prof["composite_bwd"][0] > 0
        assert all(n == 0 for k, (_, n) in prof.items() if k != "composite_bwd")
        V.profile_stages(None)
        V.profile_enable(True)
        step()
        prof = V.profile_read()
        for k in ("preprocess", "depth_sort", "tile_sort", "composite", "composite_bwd", "preprocess_bwd"):
            assert prof[k][1] >= 1, k
    finally:
        V.profile_enable(False)
        V.profile_stages(None)
