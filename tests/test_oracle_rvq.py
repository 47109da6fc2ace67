"""Pins of the R-VQ oracle (Sec. 3.4 eqs. (14)-(15)) against what the
mathematics fixes: each stage's pick is the nearest code in binary64 up to the
binary32 decision's error, the one-dimensional case is the nearest grid point,
a single 32-d stage is a k-d tree's nearest neighbour, the cascade equals
single stages applied to the residuals, a codebook that holds the inputs has a
closed-form result, and the code gradient is the finite difference of the loss
wherever no later residual depends on the code."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import rvq


def _books(rng, L, P, D, spread=1.0, decay=0.35):
    return np.stack([rng.normal(0.0, spread * decay ** l, (P, D)) for l in range(L)]).astype(np.float32)


def test_each_stage_picks_the_nearest_code():
    rng = np.random.default_rng(0)
    L, P, D, n = 4, 64, 7, 3000
    books = _books(rng, L, P, D)
    x = rng.normal(0.0, 1.0, (n, D)).astype(np.float32)
    out = rvq.rvq(books, x)
    xhat = np.zeros((n, D))
    exact = 0
    for l in range(L):
        r = x.astype(np.float64) - xhat
        d = ((books[l][None, :, :].astype(np.float64) - r[:, None, :]) ** 2).sum(-1)
        pick = out["idx"][l]
        dp = d[np.arange(n), pick]
        scale = (books[l].astype(np.float64) ** 2).sum(-1).max() + 2 * np.abs(r).sum(-1) * np.abs(books[l]).max() \
            + (r ** 2).sum(-1)
        assert np.all(dp - d.min(1) <= 1e-5 * scale + 1e-12), l
        exact += int((pick == d.argmin(1)).sum())
        xhat += books[l][pick]
    assert exact >= 0.995 * n * L
    np.testing.assert_allclose(out["recon"], xhat, rtol=0, atol=1e-5)


def test_one_dimensional_stage_is_nearest_grid_point():
    rng = np.random.default_rng(1)
    grid = np.sort(rng.uniform(-3, 3, 50)).astype(np.float32)
    x = rng.uniform(-3.5, 3.5, (4000, 1)).astype(np.float32)
    out = rvq.rvq(grid[None, :, None], x)
    g = grid.astype(np.float64)
    pos = np.clip(np.searchsorted(g, x[:, 0]), 1, len(g) - 1)
    left, right = g[pos - 1], g[pos]
    want = np.where(np.abs(x[:, 0] - left) <= np.abs(right - x[:, 0]), pos - 1, pos)
    mid = 0.5 * (left + right)
    clear = np.abs(x[:, 0] - mid) > 1e-5 * (1 + np.abs(mid))
    assert np.array_equal(out["idx"][0][clear], want[clear])


def test_single_feature_stage_is_kdtree_nearest_neighbour():
    rng = np.random.default_rng(2)
    P, D, n = 256, 32, 2000
    books = rng.normal(0.0, 1.0, (1, P, D)).astype(np.float32)
    x = (books[0][rng.integers(0, P, n)] + rng.normal(0.0, 0.6, (n, D))).astype(np.float32)
    out = rvq.rvq(books, x)
    dist, nn = cKDTree(books[0].astype(np.float64)).query(x.astype(np.float64), k=2)
    clear = (dist[:, 1] ** 2 - dist[:, 0] ** 2) > 1e-4 * (1 + dist[:, 1] ** 2)
    assert clear.mean() > 0.99
    assert np.array_equal(out["idx"][0][clear], nn[clear, 0])


def test_cascade_is_single_stages_on_residuals():
    rng = np.random.default_rng(3)
    L, P, D, n = 5, 64, 3, 1500
    books = _books(rng, L, P, D)
    x = rng.normal(0.0, 1.0, (n, D)).astype(np.float32)
    full = rvq.rvq(books, x)
    recon = np.zeros((n, D), np.float32)
    loss = 0.0
    for l in range(L):
        prev = rvq.rvq(books[:l], x)["recon"] if l > 0 else np.zeros((n, D), np.float32)
        r = (x - prev).astype(np.float32)
        one = rvq.rvq(books[l:l + 1], r)
        assert np.array_equal(one["idx"][0], full["idx"][l]), l
        np.testing.assert_allclose(one["dbooks"][0], full["dbooks"][l], rtol=1e-12, atol=1e-15)
        loss += one["loss"]
        recon = rvq.rvq(books[:l + 1], x)["recon"]
    assert loss == pytest.approx(full["loss"], rel=1e-12)
    assert np.array_equal(recon, full["recon"])


def test_codebook_holding_the_inputs():
    rng = np.random.default_rng(4)
    P, D, n = 64, 7, 40
    x = rng.normal(0.0, 1.0, (n, D)).astype(np.float32)
    b1 = rng.normal(0.0, 1.0, (P, D)).astype(np.float32)
    where = rng.permutation(P)[:n]
    b1[where] = x
    b2 = rng.normal(0.0, 0.5, (P, D)).astype(np.float32)
    k2 = int(np.argmin((b2.astype(np.float64) ** 2).sum(1)))
    out = rvq.rvq(np.stack([b1, b2]), x)
    assert np.array_equal(out["idx"][0], where)
    assert np.all(out["idx"][1] == k2)
    np.testing.assert_allclose(out["recon"], x.astype(np.float64) + b2[k2], rtol=0, atol=1e-6)
    assert out["loss"] == pytest.approx(n * float((b2[k2].astype(np.float64) ** 2).sum()) / (n * P), rel=1e-12)
    # the first stage's picked codes carry no gradient (zero residual error)
    assert np.all(out["dbooks"][0] == 0.0)
    np.testing.assert_allclose(out["dbooks"][1][k2], 2.0 * n * b2[k2].astype(np.float64) / (n * P), rtol=1e-12)


@pytest.mark.parametrize("L", [1, 3])
def test_last_stage_gradient_is_the_finite_difference(L):
    rng = np.random.default_rng(5 + L)
    P, D, n = 16, 4, 600
    books = _books(rng, L, P, D).astype(np.float64)
    x = rng.normal(0.0, 1.0, (n, D)).astype(np.float32)
    base = rvq.rvq(books, x)
    used = np.unique(base["idx"][L - 1])
    checked = 0
    for k in used[:5]:
        for j in range(D):
            h = 2.0 ** -10
            bp, bm = books.copy(), books.copy()
            bp[L - 1, k, j] += h
            bm[L - 1, k, j] -= h
            op, om = rvq.rvq(bp, x), rvq.rvq(bm, x)
            if not (np.array_equal(op["idx"], base["idx"]) and np.array_equal(om["idx"], base["idx"])):
                continue
            fd = (op["loss"] - om["loss"]) / (2 * h)
            assert fd == pytest.approx(base["dbooks"][L - 1, k, j], rel=1e-6, abs=1e-12)
            checked += 1
    assert checked >= 10


def test_empty_input():
    books = np.ones((2, 8, 3), np.float32)
    out = rvq.rvq(books, np.zeros((0, 3), np.float32))
    assert out["loss"] == 0.0 and np.all(out["dbooks"] == 0.0) and out["idx"].shape == (2, 0)


def test_equal_distances_pick_the_first_code():
    """Duplicated codes tie exactly; the pick is the lowest index, as numpy's
    argmin returns the first of equal minima."""
    rng = np.random.default_rng(12)
    P, D = 32, 5
    books = rng.normal(0.0, 1.0, (1, P, D)).astype(np.float32)
    books[0, 20] = books[0, 3]
    books[0, 29] = books[0, 11]
    x = np.concatenate([books[0, [3, 11]] + rng.normal(0.0, 1e-3, (2, D)),
                        rng.normal(0.0, 1.0, (200, D))]).astype(np.float32)
    out = rvq.rvq(books, x)
    d = ((books[0][None].astype(np.float64) - x[:, None].astype(np.float64)) ** 2).sum(-1)
    assert out["idx"][0][0] == 3 and out["idx"][0][1] == 11
    assert not np.isin(out["idx"][0], [20, 29]).any()
    assert np.array_equal(out["idx"][0], d.argmin(1))
