"""The binding refuses caller tensors that a kernel would read or write past:
wrong shapes, wrong dtypes and host tensors raise VcgsError before anything
is launched, and the library keeps working afterwards."""
import pytest
import torch

from paper_2403_11247_amd import scenes
from tests.gpu_common import dev, gauss_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    vcgs.lib()
    return vcgs


def test_wrong_shapes_and_host_tensors_are_refused(V):
    g = scenes.random_scene(500, seed=2)
    gd = gauss_dev(g)
    cam = scenes.Camera(64, 48, 50.0, 50.0, 32.0, 24.0)
    pose = scenes.identity_pose()
    C, D, A, st = V.render_forward(*gd, cam, pose)
    small_c, small_d = torch.zeros((3, 40, 64), device="cuda"), torch.zeros((40, 64), device="cuda")
    with pytest.raises(V.VcgsError):
        V.l1_loss(C, D, small_c, D)                           # target colour too small
    with pytest.raises(V.VcgsError):
        V.l1_loss(C, D, C, small_d)                           # target depth too small
    with pytest.raises(V.VcgsError):
        V.track_loss(C, D, A, C, small_d)
    with pytest.raises(V.VcgsError):
        V.ssim_loss(C, small_c)
    with pytest.raises(V.VcgsError):
        V.render_backward(st, *gd, cam, pose, small_c, None, None)   # upstream colour gradient
    with pytest.raises(V.VcgsError):
        V.icp_loss(gd[0], cam, pose, small_d)                 # observed depth not the camera's size
    with pytest.raises(V.VcgsError):
        V.icp_loss(gd[0], cam, pose, D, dpose=torch.zeros(6))  # host tensor
    with pytest.raises(V.VcgsError):
        V.render_forward(*gd, cam, pose, hits=torch.zeros(g.n, dtype=torch.int64, device="cuda"))
    with pytest.raises(V.VcgsError):
        V.add_centre_pose_grad([pose], torch.zeros((1, 3), device="cuda"), torch.zeros((1, 5), device="cuda"))
    with pytest.raises(V.VcgsError):
        V.mask_loss(dev(torch.zeros(10)), dl_dm=torch.zeros(9, device="cuda"))
    # still working
    up = [dev(x) for x in scenes.upstream_grads(cam.width, cam.height, seed=1)]
    grads, dpose = V.render_backward(st, *gd, cam, pose, *up)
    st.free()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(dpose).all())
