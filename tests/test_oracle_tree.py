"""Pins of the oracle tree (Alg. 2) and prediction (CPU only)."""
import numpy as np
import pytest

from oracle import pso as O
from oracle import split as S
from oracle import tree as T
from paper_2208_07023_amd import inputs


def test_depth_one_tree_is_the_root_swarm():
    X, y, _ = inputs.two_class_gaussian(300, 4, seed=3)
    prm = T.TreeParams(crit=S.GINI, K=2, max_depth=1, min_node=2, P=8, T=5, bins=32, seed=4)
    tr = T.grow_tree(X, y, prm)
    res = O.run_pso(T.evaluate_node(X, y, prm), 8, 4, 5, 0.7, 1.5, 1.5, 4, 0, 0)
    A = tr.arrays()
    assert len(A["thr"]) == 3
    assert np.array_equal(A["w"][0], res["gbest"].astype(np.float32))
    assert A["thr"][0] == res["thr"] and A["split_loss"][0] == res["loss"]
    z = S.project(X, A["w"][:1]).astype(np.float32)[:, 0]
    assert A["n"][1] == int((z < A["thr"][0]).sum()) and A["n"][1] + A["n"][2] == 300
    # the histogram split's left count is the chosen bin boundary
    b = S.hist_bins(z, z.min(), z.max(), 32)
    assert A["n"][1] == int((b < res["split"]).sum())


def test_pure_and_small_nodes_are_leaves():
    X, _, _ = inputs.two_class_gaussian(100, 3, seed=1)
    y = np.zeros(100, dtype=np.int32)
    tr = T.grow_tree(X, y, T.TreeParams(crit=S.GINI, K=2, P=4, T=2))
    assert len(tr.thr) == 1 and tr.left[0] == -1
    y[:3] = 1
    tr = T.grow_tree(X, y, T.TreeParams(crit=S.GINI, K=2, P=4, T=2, min_node=101))
    assert len(tr.thr) == 1


def test_tree_structure_invariants():
    X, y = inputs.cluster_mixture(3000, 8, 3, seed=5)
    prm = T.TreeParams(crit=S.ENTROPY, K=3, max_depth=4, min_node=32, P=16, T=6, bins=64, seed=1)
    tr = T.grow_tree(X, y, prm, keep_rows=True)
    A = tr.arrays()
    assert A["depth"].max() <= 4
    for i in range(len(A["thr"])):
        if A["left"][i] >= 0:
            l, r = A["left"][i], A["right"][i]
            assert A["heap"][l] == 2 * A["heap"][i] + 1 and A["heap"][r] == 2 * A["heap"][i] + 2
            assert np.array_equal(np.sort(np.concatenate([tr.rows[l], tr.rows[r]])), np.sort(tr.rows[i]))
            assert A["n"][i] >= 32 and A["split_loss"][i] < A["impurity"][i]
            # children are weighted-impurity consistent with the split loss
            wimp = (A["n"][l] * A["impurity"][l] + A["n"][r] * A["impurity"][r]) / A["n"][i]
            assert wimp == pytest.approx(A["split_loss"][i], rel=1e-9, abs=1e-12)
    # breadth-first order: depths non-decreasing
    assert np.all(np.diff(A["depth"]) >= 0)


def test_classification_accuracy_near_bayes():
    """Identity covariance: Bayes accuracy is Phi(||mu1 - mu0|| / 2)."""
    from scipy.stats import norm
    Xa, ya, means = inputs.two_class_gaussian(4000, 8, seed=7)
    X, y, Xt, yt = Xa[:2000], ya[:2000], Xa[2000:], ya[2000:]     # held-out half
    tr = T.grow_tree(X, y, T.TreeParams(crit=S.GINI, K=2, max_depth=3, P=32, T=10, bins=256))
    acc = float((T.predict(tr, Xt) == yt).mean())
    bayes = norm.cdf(np.linalg.norm(means[1] - means[0]) / 2)
    assert bayes - 0.04 < acc <= bayes + 0.03


def test_regression_tree_beats_the_mean():
    X, y = inputs.abs_direction_regression(4000, 8, n_dirs=2, seed=2)
    tr = T.grow_tree(X, y, T.TreeParams(crit=S.MSE, K=0, max_depth=4, P=16, T=8, bins=64))
    pred = T.predict(tr, X)
    assert np.mean((pred - y) ** 2) < 0.6 * np.var(y)
    A = tr.arrays()
    assert A["leaf"][0][0] == pytest.approx(y.mean(), rel=1e-12)
