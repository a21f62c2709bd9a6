"""Pins of the forest and boosting oracle (oracle.ensemble; CPU only).

* bootstrap draws: the law of sampling N rows with replacement (distinct-row
  fraction 1 - (1 - 1/N)^N, multiplicities Poisson(1) in the limit, uniform
  rows), the top-bits form of the row map when N is a power of two, and
  independence across tree ids;
* forest: a one-tree forest without bootstrap is the plain tree; every tree is
  the plain tree of its sample; hand-counted votes and means; the convexity
  bound of the mean aggregate (the forest's squared error never exceeds the
  trees' mean squared error, at every point);
* boosting: the exact training-error recursion of a squared-loss round with
  leaf means (SSE' = SSE - (2 lr - lr^2) sum_l n_l m_l^2), the closed-form
  first softmax round of a stump, and a decreasing training log-loss.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import ensemble as E
from oracle import philox as PH
from oracle import split as S
from oracle import tree as T
from paper_2208_07023_amd import inputs


# ---------------------------------------------------------------- bootstrap
def test_bootstrap_follows_sampling_with_replacement():
    N = 100_000
    for tree in (0, 7):
        idx = E.bootstrap_indices(11, tree, N)
        assert idx.shape == (N,) and idx.min() >= 0 and idx.max() < N
        cnt = np.bincount(idx, minlength=N)
        # distinct fraction: 1 - (1 - 1/N)^N, sd ~ 1e-3
        assert abs((cnt > 0).mean() - (1 - (1 - 1 / N) ** N)) < 0.004
        # multiplicities ~ Poisson(1): P(k) = e^-1 / k!
        for k in range(4):
            p = math.exp(-1) / math.factorial(k)
            assert abs((cnt == k).mean() - p) < 4 * math.sqrt(p * (1 - p) / N) + 1e-3, k
        # uniform rows: mean index (N - 1) / 2, sd N / sqrt(12 N)
        assert abs(idx.mean() - (N - 1) / 2) < 4 * N / math.sqrt(12 * N)
        # decile counts
        dec = np.bincount(idx * 10 // N, minlength=10)
        assert np.all(np.abs(dec - N / 10) < 4 * math.sqrt(N * 0.09))


def test_bootstrap_power_of_two_takes_the_top_bits():
    N = 1 << 12
    idx = E.bootstrap_indices(5, 3, N)
    ctr = np.zeros((N // 4, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(N // 4)
    ctr[:, 1] = E.BOOT_STREAM
    ctr[:, 2] = E.NO_NODE
    ctr[:, 3] = 3
    w = PH.philox4x32_10(ctr, PH.seed_key(5)).reshape(-1)
    assert np.array_equal(idx, (w >> np.uint32(20)).astype(np.int64))


def test_bootstrap_edges_and_independence():
    assert E.bootstrap_indices(1, 0, 0).shape == (0,)
    assert np.array_equal(E.bootstrap_indices(1, 0, 1), [0])
    # a ragged tail (N not a multiple of 4) is a prefix of the longer draw's words
    a = E.bootstrap_indices(1, 2, 7)
    assert a.shape == (7,) and a.max() < 7
    assert np.array_equal(a, E.bootstrap_indices(1, 2, 7))
    N = 50_000
    s0 = np.unique(E.bootstrap_indices(2, 0, N))
    s1 = np.unique(E.bootstrap_indices(2, 1, N))
    s2 = np.unique(E.bootstrap_indices(3, 0, N))
    q = 1 - (1 - 1 / N) ** N
    for u in (s1, s2):
        # independent samples share q^2 of the rows
        assert abs(np.intersect1d(s0, u).size / N - q * q) < 0.01


# ---------------------------------------------------------------- forest
def _prm(**kw):
    base = dict(crit=S.GINI, K=3, max_depth=3, min_node=8, P=8, T=4, bins=32, seed=5)
    base.update(kw)
    return T.TreeParams(**base)


def test_one_tree_forest_without_bootstrap_is_the_tree():
    X, y = inputs.cluster_mixture(400, 5, 3, seed=1)
    prm = _prm()
    f = E.grow_forest(X, y, prm, 1, bootstrap=False)
    a, b = f.trees[0].arrays(), T.grow_tree(X, y, prm).arrays()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_forest_trees_are_the_trees_of_their_samples():
    X, y = inputs.cluster_mixture(300, 4, 3, seed=2)
    prm = _prm(tree=10)
    f = E.grow_forest(X, y, prm, 3)
    for b, (tr, idx) in enumerate(zip(f.trees, f.samples)):
        assert np.array_equal(idx, E.bootstrap_indices(prm.seed, 10 + b, 300))
        ref = T.grow_tree(X[idx], y[idx], dataclasses.replace(prm, tree=10 + b)).arrays()
        got = tr.arrays()
        for k in got:
            assert np.array_equal(got[k], ref[k]), (b, k)
        # the root holds the bootstrap sample's class counts
        assert np.array_equal(got["leaf"][0], np.bincount(y[idx], minlength=3))
    # different trees saw different samples
    assert not np.array_equal(f.samples[0], f.samples[1])


def test_combine_votes_and_means_by_hand():
    out = np.array([[0, 2, 1, 1, 2],
                    [2, 2, 0, 1, 0],
                    [1, 0, 0, 1, 1]])
    # row 0: one vote each -> 0; row 1: 2 wins; row 2: 0 twice; row 3: all 1;
    # row 4: one vote each -> 0
    assert np.array_equal(E.combine(out, 3), [0, 2, 0, 1, 0])
    # a class nobody votes for never wins; K larger than the votes seen
    assert np.array_equal(E.combine(np.array([[3], [3], [1]]), 5), [3])
    reg = np.array([[1.0, -2.0], [2.0, 4.0], [4.5, 1.0]])
    assert np.array_equal(E.combine(reg, 0), [7.5 / 3, 1.0])


def test_regression_forest_never_exceeds_mean_tree_error():
    X, y = inputs.friedman1(600, 6, noise=1.0, seed=3)
    prm = _prm(crit=S.MSE, K=0, max_depth=4, bins=32)
    f = E.grow_forest(X, y, prm, 4)
    Xt, yt = inputs.friedman1(300, 6, noise=1.0, seed=4)
    outs = E.tree_outputs(f, Xt)
    pred = E.forest_predict(f, Xt)
    assert np.allclose(pred, outs.mean(axis=0), rtol=0, atol=1e-12)
    err_f = (pred - yt) ** 2
    err_t = ((outs - yt) ** 2).mean(axis=0)
    assert np.all(err_f <= err_t + 1e-9)
    # and strictly on average once the trees disagree
    assert err_f.mean() < err_t.mean()


def test_classification_forest_output_is_a_voted_class():
    X, y = inputs.cluster_mixture(400, 5, 3, seed=6)
    f = E.grow_forest(X, y, _prm(), 5)
    Xt, _ = inputs.cluster_mixture(200, 5, 3, seed=7)
    outs = E.tree_outputs(f, Xt)
    pred = E.forest_predict(f, Xt)
    for i in range(Xt.shape[0]):
        assert pred[i] in outs[:, i]
        c = np.bincount(outs[:, i], minlength=3)
        assert c[pred[i]] == c.max() and np.all(c[:pred[i]] < c.max())


# ---------------------------------------------------------------- boosting
def test_squared_loss_round_lowers_sse_by_the_leaf_means():
    X, y = inputs.friedman1(500, 6, noise=0.5, seed=8)
    prm = _prm(crit=S.MSE, K=0, max_depth=3, bins=32)
    for lr in (1.0, 0.3):
        model, F = E.boost_regression(X, y, prm, 3, lr)
        assert F[0][0] == pytest.approx(y.mean(), rel=1e-15)
        for m, tr in enumerate(model.trees):
            A = tr.arrays()
            leaves = A["left"] < 0
            n_l, m_l = A["n"][leaves], A["leaf"][leaves, 0]
            sse0 = np.sum((y - F[m]) ** 2)
            sse1 = np.sum((y - F[m + 1]) ** 2)
            assert sse1 == pytest.approx(sse0 - (2 * lr - lr * lr) * np.sum(n_l * m_l ** 2),
                                         rel=1e-9)
            assert sse1 < sse0
        # scoring from the model reproduces the training trajectory
        assert np.allclose(E.boost_scores(model, X), F[-1], rtol=0, atol=1e-12)


def test_softmax_stump_round_in_closed_form():
    X, y = inputs.cluster_mixture(300, 4, 3, seed=9)
    y = y.copy()
    y[:40] = 0          # unequal class frequencies
    prm = _prm(max_depth=0)
    model, F = E.boost_classification(X, y, 3, prm, 2, 0.5)
    pi = np.bincount(y, minlength=3) / y.size
    assert np.allclose(F[1], np.tile(0.5 * (pi - 1 / 3), (300, 1)), rtol=0, atol=1e-15)
    # second round: p = softmax(F_1), step = mean of the residuals
    p = E.softmax(F[1])
    step = (np.eye(3)[y] - p).mean(axis=0)
    assert np.allclose(F[2], F[1] + 0.5 * step, rtol=0, atol=1e-15)


def test_softmax_boost_lowers_training_log_loss():
    X, y = inputs.cluster_mixture(600, 5, 3, seed=10)
    prm = _prm(max_depth=3, T=6)
    model, F = E.boost_classification(X, y, 3, prm, 4, 0.3)
    ll = [-np.mean(np.log(E.softmax(f)[np.arange(y.size), y])) for f in F]
    assert ll[0] == pytest.approx(math.log(3), rel=1e-15)
    assert all(b < a for a, b in zip(ll, ll[1:])), ll
    assert np.array_equal(E.boost_predict(model, X), np.argmax(F[-1], axis=1))
    acc = (E.boost_predict(model, X) == y).mean()
    assert acc > 0.6
