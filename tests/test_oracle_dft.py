"""Pins of the DFT / top-n channel oracle (Alg. 2) against facts that do not
depend on its own code: a perfectly separating feature, brute-force best
thresholds in exact arithmetic, the ordering rule, the geometry of the
restricted start, invariance of the restriction under swarm moves, and the
special cases n = D (the plain tree) and n = 1 (axis-aligned splits)."""
import numpy as np
import pytest

from oracle import brute, dft, pso, split as S, tree as OT


def _separable(n, D, K, col, seed):
    rng = np.random.default_rng(seed)
    y = rng.integers(0, K, n).astype(np.int32)
    X = rng.uniform(-1, 1, (n, D)).astype(np.float32)
    X[:, col] = (y * 4.0 + rng.uniform(0, 1, n)).astype(np.float32)   # disjoint per class
    return X, y


@pytest.mark.parametrize("crit", [S.GINI, S.ENTROPY])
@pytest.mark.parametrize("bins", [0, 64])
def test_separating_feature_has_zero_loss_and_is_selected_first(crit, bins):
    X, y = _separable(400, 6, 2, col=4, seed=1)
    loss = dft.dft_losses(X, y, crit, 2, bins)
    assert loss[4] == 0.0
    assert np.all(np.delete(loss, 4) > 0.05)
    assert list(dft.top_n(loss, 1)) == [4]


@pytest.mark.parametrize("crit,K", [(S.GINI, 2), (S.ENTROPY, 3)])
def test_exact_dft_losses_equal_brute_force_best_thresholds(crit, K):
    rng = np.random.default_rng(7)
    X = rng.integers(-3, 4, (14, 3)).astype(np.float32)   # ties between values
    y = rng.integers(0, K, 14).astype(np.int32)
    loss = dft.dft_losses(X, y, crit, K, 0)
    for d in range(3):
        ts = np.unique(X[:, d])
        _, best, _ = brute.best_over(X[:, d], y, ts, crit, K)
        if best is None:
            assert np.isposinf(loss[d])
        else:
            assert loss[d] == pytest.approx(float(best), rel=1e-13, abs=1e-15)


def test_top_n_order_ties_and_no_split_last():
    loss = np.array([1.0, 0.5, 0.5, np.inf, 0.2, 0.5])
    assert list(dft.top_n(loss, 4)) == [4, 1, 2, 5]
    assert list(dft.top_n(loss, 6)) == [4, 1, 2, 5, 0, 3]


def test_subspace_start_geometry():
    P, D = 9, 7
    sel = [5, 1, 3]
    x = dft.subspace_start(3, 2, 11, P, D, sel)
    out = np.setdiff1d(np.arange(D), sel)
    assert np.all(x[:, out] == 0.0)
    assert np.allclose(np.linalg.norm(x, axis=1), 1.0, rtol=0, atol=4e-16)
    # all channels: the plain start, bit for bit
    assert np.array_equal(dft.subspace_start(3, 2, 11, P, D, np.arange(D)),
                          pso.init_positions(3, 2, 11, P, D))
    # one channel: +-e_d
    x1 = dft.subspace_start(3, 2, 11, P, D, [4])
    assert np.all(np.abs(x1[:, 4]) == 1.0) and np.all(np.delete(x1, 4, axis=1) == 0.0)


def test_moves_stay_in_the_subspace():
    P, D = 16, 6
    sel = [0, 2, 5]
    x = dft.subspace_start(1, 0, 3, P, D, sel)
    v = np.zeros_like(x)
    pb, pbl = x.copy(), np.full(P, np.inf)
    gb, gbl, gp = x[:1].copy(), np.array([np.inf]), np.array([-1])
    rng = np.random.default_rng(0)
    for it in range(1, 8):
        loss = rng.uniform(0, 1, P)
        out = pso.pso_step(x, v, pb, pbl, gb, gbl, gp, loss, np.array([3]), 1, P, D,
                           0.7, 1.5, 1.5, 1, 0, it, True)
        x, v, pb, pbl = out["x"], out["v"], out["pbest"], out["pbest_loss"]
        gb, gbl, gp = out["gbest"], out["gbest_loss"], out["gbest_p"]
        for a in (x, v, pb, gb):
            assert np.all(a[:, [1, 3, 4]] == 0.0)
        assert np.allclose(np.linalg.norm(x, axis=1), 1.0, rtol=0, atol=4e-16)


def _data(n, D, K, seed):
    rng = np.random.default_rng(seed)
    y = rng.integers(0, K, n).astype(np.int32)
    means = rng.normal(0, 1.5, (K, D))
    return (means[y] + rng.normal(0, 1, (n, D))).astype(np.float32), y


def test_tree_with_all_channels_is_the_plain_tree():
    X, y = _data(300, 5, 3, seed=2)
    base = dict(crit=S.GINI, K=3, max_depth=3, min_node=20, P=8, T=4, bins=32, seed=5)
    a = OT.grow_tree(X, y, OT.TreeParams(**base)).arrays()
    b = OT.grow_tree(X, y, OT.TreeParams(dft_top_n=5, **base)).arrays()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("crit", [S.GINI, S.ENTROPY])
def test_one_channel_tree_splits_on_the_best_dft_feature(crit):
    X, y = _data(60, 4, 2, seed=4)
    prm = OT.TreeParams(crit=crit, K=2, max_depth=1, min_node=10, P=8, T=3, bins=16, seed=1,
                        dft_top_n=1)
    tr = OT.grow_tree(X, y, prm).arrays()
    loss = dft.dft_losses(X, y, crit, 2, 16)
    d = int(dft.top_n(loss, 1)[0])
    w = tr["w"][0]
    assert np.count_nonzero(w) == 1 and abs(w[d]) == 1.0
    # the split is a threshold on x_d: between the best over all thresholds
    # (exact, brute force) and the histogram DFT loss of x_d
    ts = np.unique(X[:, d])
    _, best, _ = brute.best_over(X[:, d], y, ts, crit, 2)
    assert float(best) - 1e-12 <= tr["split_loss"][0] <= loss[d] + 1e-15
