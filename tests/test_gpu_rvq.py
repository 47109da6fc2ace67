"""Residual vector quantization on the GPU (Sec. 3.4 eqs. (14)-(15)) against
the oracle: code indices and reconstructions bit for bit (the nearest-code
decision is binary32 on both sides, in the same order), the loss within 1e-5
and the code gradient within 1e-3 relative; the paper's variants (64 codes x
4 or 6 stages on anchor scaling and offsets, per-Gaussian scale and rotation,
256-code one-byte feature books), ragged and degenerate sizes, index width,
gradient accumulation and the argument checks."""
import numpy as np
import pytest
import torch

from oracle import rvq as orvq
from paper_2403_11247_amd import scenes
from tests.gpu_common import dev, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_2403_11247_amd import vcgs
    vcgs.lib()
    return vcgs


def check(V, books, x, idx_bytes=1, grad=True):
    ref = orvq.rvq(books, x)
    out = V.rvq_assign(dev(books), dev(x), idx_bytes=idx_bytes, grad=grad)
    torch.cuda.synchronize()
    idx = out["idx"].cpu().numpy().astype(np.int64)
    assert np.array_equal(idx, ref["idx"]), np.argwhere(idx != ref["idx"])[:5]
    assert np.array_equal(out["recon"].cpu().numpy(), ref["recon"])
    loss = float(out["loss"][0])
    assert abs(loss - ref["loss"]) <= 1e-5 * abs(ref["loss"]) + 1e-30, (loss, ref["loss"])
    if grad:
        g = out["dbooks"].cpu().numpy().astype(np.float64)
        r = ref["dbooks"]
        scale = np.abs(r).max() + 1e-30
        assert np.all(np.abs(g - r) <= 1e-3 * np.abs(r) + 1e-5 * scale), np.abs(g - r).max() / scale
    return out, ref


@pytest.mark.parametrize("kind,n,L,P", [
    ("scaling", 40_000, 6, 64),   # anchor scaling, the paper's 6 stages
    ("offset", 10_007, 4, 64),    # anchor offsets, the ablation's 4 stages
    ("gauss", 100_003, 6, 64),    # per-Gaussian log-scale + rotation
    ("feature", 40_000, 1, 256),  # one-byte anchor feature codes
])
def test_paper_variants(V, kind, n, L, P):
    books, x = scenes.rvq_problem(kind, n, L, P, seed=n)
    out, ref = check(V, books, x)
    used = len(np.unique(ref["idx"][0]))
    say(f"rvq {kind}: n={n} L={L} P={P} loss {ref['loss']:.4e}, stage-1 codes used {used}")


@pytest.mark.parametrize("L,P,D,n", [(3, 5, 3, 1000), (2, 1, 1, 77), (1, 3, 17, 130), (1, 200, 32, 65),
                                     (8, 7, 9, 3)])
def test_ragged_and_degenerate(V, L, P, D, n):
    rng = np.random.default_rng(L * 100 + P)
    books = rng.normal(0.0, 1.0, (L, P, D)).astype(np.float32)
    x = rng.normal(0.0, 1.0, (n, D)).astype(np.float32)
    check(V, books, x)


def test_max_stages_and_codes_without_gradient(V):
    books, x = scenes.rvq_problem("scaling", 20_000, 8, 256, seed=3)
    check(V, books, x, grad=False)


def test_index_width_ties_and_accumulation(V):
    rng = np.random.default_rng(9)
    books = rng.normal(0.0, 1.0, (2, 64, 4)).astype(np.float32)
    books[0, 40] = books[0, 7]  # duplicate code: the first index wins
    x = np.concatenate([np.repeat(books[0, 7][None], 50, 0), rng.normal(0.0, 1.0, (5000, 4))]).astype(np.float32)
    o1, ref = check(V, books, x, idx_bytes=1)
    o4, _ = check(V, books, x, idx_bytes=4)
    assert torch.equal(o1["idx"].int(), o4["idx"])
    assert np.all(ref["idx"][0][:50] == 7)
    base = torch.randn(2, 64, 4, device="cuda")
    o = V.rvq_assign(dev(books), dev(x), dbooks=base.clone(), grad=True)
    # added to what dbooks held: one rounding of the sum, plus the code sums' own order
    got = o["dbooks"].cpu().numpy().astype(np.float64)
    want = base.cpu().numpy().astype(np.float64) + o1["dbooks"].cpu().numpy()
    assert np.all(np.abs(got - want) <= np.spacing(np.abs(want).astype(np.float32)) + 1e-4 * np.abs(
        o1["dbooks"].cpu().numpy()))


def test_empty_and_rejections(V):
    books = torch.ones(2, 8, 3, device="cuda")
    out = V.rvq_assign(books, torch.zeros(0, 3, device="cuda"), grad=True)
    torch.cuda.synchronize()
    assert float(out["loss"][0]) == 0.0 and float(out["dbooks"].abs().max()) == 0.0
    with pytest.raises(V.VcgsError):
        V.rvq_assign(torch.ones(1, 257, 3, device="cuda"), torch.zeros(4, 3, device="cuda"))
    with pytest.raises(V.VcgsError):
        V.rvq_assign(torch.ones(8, 256, 32, device="cuda"), torch.zeros(4, 32, device="cuda"), grad=True)
    with pytest.raises(V.VcgsError):
        V.rvq_assign(torch.ones(1, 8, 33, device="cuda"), torch.zeros(4, 33, device="cuda"))


def test_code_gradient_is_bit_reproducible(V):
    """The per-block code sums are exact integers, so repeated calls give the
    same bits for every output, the code gradient included."""
    books, x = scenes.rvq_problem("gauss", 200_000, 6, 64, seed=4)
    outs = [V.rvq_assign(dev(books), dev(x), grad=True) for _ in range(3)]
    torch.cuda.synchronize()
    for o in outs[1:]:
        for k in ("idx", "recon", "loss", "dbooks"):
            assert torch.equal(o[k], outs[0][k]), k


def test_codebooks_learn_from_the_code_gradient(V):
    """Codebooks trained on eq. (15) with the GPU gradient (Adam, 60 steps)
    lower the quantisation loss and the reconstruction error of the
    per-Gaussian (log-scale, rotation) vectors; the assignment follows them."""
    books, x = scenes.rvq_problem("gauss", 50_000, 4, 64, seed=8)
    b = dev(books)
    xx = dev(x)
    opt = torch.optim.Adam([b.requires_grad_()], lr=2e-3)
    first = None
    for it in range(60):
        out = V.rvq_assign(b.detach(), xx, grad=True)
        loss = float(out["loss"][0])
        first = loss if first is None else first
        opt.zero_grad()
        b.grad = out["dbooks"]
        opt.step()
    final = V.rvq_assign(b.detach(), xx)
    err0 = float(((V.rvq_assign(dev(books), xx)["recon"] - xx) ** 2).mean())
    err1 = float(((final["recon"] - xx) ** 2).mean())
    say(f"rvq fit: loss {first:.4e} -> {float(final['loss'][0]):.4e}, recon mse {err0:.3e} -> {err1:.3e}")
    assert float(final["loss"][0]) < 0.8 * first
    assert err1 < 0.5 * err0
