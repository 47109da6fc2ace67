"""The allocation-free forward render (vcgs_render_forward_noalloc) against the
plain forward (vcgs_render_forward): the same kernels on the same inputs, so
the images must agree bit for bit -- on two calls in a row, the second with a
smaller scene and a ragged image, on the room workload (400k Gaussians,
1200x680), and after a call that the scratch array could not hold."""
import numpy as np
import pytest
import torch

from paper_2403_11247_amd import scenes
from tests.gpu_common import FIELDS, dev, gauss_dev, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    vcgs.lib()
    return vcgs


def _outs(cam, fill=float("nan")):
    H, W = cam.height, cam.width
    return (torch.full((3, H, W), fill, device="cuda"), torch.full((H, W), fill, device="cuda"),
            torch.full((H, W), fill, device="cuda"))


def _same(V, gd, cam, pose, bg=(0.0, 0.0, 0.0)):
    C, D, A, _ = V.render_forward(*gd, cam, pose, bg=bg, keep_state=False)
    out = _outs(cam)
    V.render_forward_noalloc(*gd, cam, pose, out, bg=bg)
    torch.cuda.synchronize()
    for name, a, b in zip(("colour", "depth", "alpha"), out, (C, D, A)):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"{name} differs from the plain forward"
    return out


def test_two_calls_second_smaller(V):
    say("noalloc: 2000 Gaussians 128x96, then 300 Gaussians 77x45")
    g = scenes.random_scene(2000, seed=0)
    _same(V, gauss_dev(g), scenes.random_camera(), scenes.identity_pose(), bg=(0.1, 0.2, 0.3))
    small = scenes.random_scene(300, seed=4)
    cam = scenes.Camera(77, 45, 60.0, 60.0, 38.0, 22.0)
    _same(V, gauss_dev(small), cam, scenes.perturb_pose(scenes.identity_pose(), 1, trans=0.05, rot_deg=3.0))


def test_room_fits_and_matches(V):
    say("noalloc: room 400k Gaussians 1200x680")
    from oracle import decode as odec
    dec = odec.decode(scenes.room_anchors(40000, k=10), scenes.room_mlp())
    gd = [dev(dec[f].astype(np.float32)) for f in FIELDS]
    cam, pose = scenes.room_camera()
    _same(V, gd, cam, pose)
    # and a smaller call right after it on the same array
    _same(V, [t[..., :5000].contiguous() for t in gd], scenes.Camera(320, 240, 160.0, 160.0, 160.0, 120.0), pose)


def test_empty_map_gives_background(V):
    say("noalloc: empty map")
    gd = [torch.empty(s, device="cuda") for s in ((3, 0), (3, 0), (4, 0), (0,), (3, 0))]
    cam = scenes.random_camera()
    out = _same(V, gd, cam, scenes.identity_pose(), bg=(0.25, 0.5, 0.75))
    assert torch.all(out[0][1] == 0.5) and torch.all(out[2] == 0.0)


def test_too_large_is_refused_and_the_next_call_works(V):
    # pairs: 20k Gaussians, each covering all 1200 tiles of a 640x480 view,
    # need 24M (tile, Gaussian) pairs -- far beyond the 128 MiB array
    say("noalloc: 24M pairs refused")
    n = 20000
    rng = np.random.default_rng(7)
    mean = np.stack([rng.uniform(-0.1, 0.1, n), rng.uniform(-0.1, 0.1, n), rng.uniform(2.0, 3.0, n)])
    big = scenes.Gaussians(mean.astype(np.float32), np.full((3, n), 5.0, np.float32),
                           np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)),
                           np.full(n, 0.5, np.float32), np.full((3, n), 0.5, np.float32))
    cam = scenes.Camera(640, 480, 320.0, 320.0, 320.0, 240.0)
    out = _outs(cam)
    with pytest.raises(V.VcgsError, match="error -3"):
        V.render_forward_noalloc(*gauss_dev(big), cam, scenes.identity_pose(), out)
    assert V.last_required_pairs() == n * 40 * 30
    torch.cuda.synchronize()
    assert torch.isnan(out[0]).all(), "a refused call left the images unwritten"
    # Gaussians: 2M entries need about 200 MB before any pair; refused before launch
    say("noalloc: 2M Gaussians refused")
    m = 2_000_000
    huge = [torch.zeros(s, device="cuda") for s in ((3, m), (3, m), (4, m), (m,), (3, m))]
    with pytest.raises(V.VcgsError, match="error -3"):
        V.render_forward_noalloc(*huge, cam, scenes.identity_pose(), out)
    del huge
    # the array still serves a normal call
    _same(V, gauss_dev(scenes.random_scene(2000, seed=3)), scenes.random_camera(), scenes.identity_pose())


def test_outputs_are_checked(V):
    g = gauss_dev(scenes.random_scene(100, seed=0))
    cam = scenes.random_camera()
    with pytest.raises(V.VcgsError):
        V.render_forward_noalloc(*g, cam, scenes.identity_pose(), _outs(scenes.Camera(64, 48, 1.0, 1.0, 1.0, 1.0)))
