"""The compacted room (mask + residual codebooks, Sec. 3.3-3.4): with 2-stage
residual k-means codebooks of 4096 x 7 fit to the room's decoded
(log-scale, quaternion) and mask logits N(2, 1), the decoded map renders
close to the unquantized one (PSNR bound below), the decode reproduces the
codebook sums it was given, and a forward + backward step gives finite
codebook and mask gradients that reach the used rows only."""
import numpy as np
import pytest
import torch

from paper_2403_11247_amd import scenes
from tests.gpu_common import FIELDS, dev, say

pytestmark = pytest.mark.gpu

PSNR_MIN_DB = 38.0  # colour PSNR of the compacted render against the unquantized one (measured 42.3)


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    vcgs.lib()
    return vcgs


def test_compacted_room_matches_unquantized(V):
    from paper_2403_11247_amd import codebook_fit
    a = scenes.room_anchors(40000, k=10)
    m = scenes.room_mlp(seed=0)
    n = a.n * a.k
    A = [dev(x) for x in (a.xa, a.feat, a.scaling, a.offset, m.W1, m.b1, m.W2, m.b2)]
    G0 = V.decode_anchors(*A)
    x = codebook_fit.shape_vectors(G0)
    books, idx = codebook_fit.residual_kmeans(x, stages=2, size=4096, iters=6)
    mask, _, _ = scenes.mask_and_codebook(n)
    ml = dev(mask)
    Gq = V.decode_anchors(*A, books=books, idx=idx, mask_logit=ml)
    torch.cuda.synchronize()
    # the decode gathers the codebook sums it was given: log-scale and quaternion
    il = idx.long()
    want = books[0][il[0]] + books[1][il[1]]
    keep = (torch.sigmoid(ml) > 0.01)
    got_ls = torch.log(Gq["scale"][:, keep]).t()
    assert torch.allclose(got_ls, want[keep][:, :3], rtol=0, atol=1e-5)
    assert torch.equal(Gq["quat"].t(), want[:, 3:])
    cam, pose = scenes.room_camera()
    C0, D0, _, _ = V.render_forward(*[G0[f] for f in FIELDS], cam, pose, keep_state=False)
    Cq, Dq, _, _ = V.render_forward(*[Gq[f] for f in FIELDS], cam, pose, keep_state=False)
    torch.cuda.synchronize()
    p = codebook_fit.psnr(Cq.clamp(0, 1), C0.clamp(0, 1))
    say(f"compacted room: colour PSNR {p:.2f} dB, depth MAE {float((Dq - D0).abs().mean()):.4f} m, "
        f"kept {int(keep.sum())} of {n}")
    assert p >= PSNR_MIN_DB, p
    # one step with codebook and mask gradients
    tC, tD, _, _ = V.render_forward(*[Gq[f] for f in FIELDS], cam, scenes.perturb_pose(pose, 2), keep_state=False)
    C, D, _, st = V.render_forward(*[Gq[f] for f in FIELDS], cam, pose)
    _, dlc, dld = V.l1_loss(C, D, tC, tD, 0.5)
    grads, dpose = V.render_backward(st, *[Gq[f] for f in FIELDS], cam, pose, dlc, dld, None)
    ag = V.decode_anchors_backward(*A, grads, books=books, idx=idx, mask_logit=ml)
    st.free()
    torch.cuda.synchronize()
    for k in ("books", "mask_logit", "feat", "W1", "W2"):
        assert bool(torch.isfinite(ag[k]).all()), k
    used = torch.zeros(2, 4096, dtype=torch.bool, device=books.device)
    used[0, il[0]] = True
    used[1, il[1]] = True
    assert bool((ag["books"][~used] == 0).all())
    assert float(ag["books"].abs().sum()) > 0 and bool(torch.isfinite(dpose).all())
