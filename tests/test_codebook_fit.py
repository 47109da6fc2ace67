"""The compacted room's input preparation (residual k-means codebooks,
paper_2403_11247_amd/codebook_fit.py), on the CPU: data with no more distinct
rows than codes is reproduced, a second stage lowers the error, every index
is in range and picks a nearest code, and the PSNR helper matches its
definition."""
import math

import numpy as np
import torch

from paper_2403_11247_amd import codebook_fit


def test_distinct_rows_are_reproduced():
    # 12 distinct rows, 128 codes drawn from the data: every row seeds a code
    # (for this seed), and Lloyd steps keep codes on their rows
    rng = np.random.default_rng(0)
    protos = torch.as_tensor(rng.normal(size=(12, 7)), dtype=torch.float32)
    x = protos[torch.as_tensor(rng.integers(0, 12, 600))]
    books, idx = codebook_fit.residual_kmeans(x, stages=1, size=128, iters=5, seed=1)
    rec = books[0][idx[0].long()]
    assert float((rec - x).abs().max()) < 1e-5


def test_second_stage_lowers_error_and_indices_in_range():
    rng = np.random.default_rng(2)
    x = torch.as_tensor(rng.normal(size=(3000, 7)), dtype=torch.float32)
    books, idx = codebook_fit.residual_kmeans(x, stages=2, size=64, iters=8, seed=3)
    assert books.shape == (2, 64, 7) and idx.shape == (2, 3000) and idx.dtype == torch.int32
    assert int(idx.min()) >= 0 and int(idx.max()) < 64
    il = idx.long()
    e1 = float(((books[0][il[0]] - x) ** 2).sum(1).mean())
    e2 = float(((books[0][il[0]] + books[1][il[1]] - x) ** 2).sum(1).mean())
    assert e2 < 0.9 * e1
    # each stage's index is the nearest code of the residual it quantises
    r = x - books[0][il[0]]
    d = ((r[:, None, :] - books[1][None, :, :]) ** 2).sum(2)
    gap = d.gather(1, il[1][:, None]) - d.min(1, keepdim=True).values
    assert float(gap.max()) < 1e-5


def test_psnr_definition():
    a = torch.zeros(3, 4, 5)
    b = torch.full((3, 4, 5), 0.1)
    assert abs(codebook_fit.psnr(a, b) - 20.0) < 1e-4  # 10 log10(1 / 0.01)
    assert math.isinf(codebook_fit.psnr(a, a))
