"""Oracle: SLM/SLR Forest (bagging) and SLM/SLR Boost (boosting) of SLM trees
(Sec. V, benchmarking settings; 30 trees per ensemble in the paper's runs).

The paper names the two ensembles, says they follow random forests (bagging)
and XGBoost (boosting) for decision trees, fixes 30 trees, and leaves the rest
to its reference.  Readings of this build:

Forest
* tree b of a forest of B trees (b = 0 .. B-1) is an SLM tree (oracle.tree)
  with tree id tree0 + b, grown on a bootstrap sample of the N rows: N draws
  with replacement, uniform over the rows (Breiman's bagging), kept in draw
  order; without bootstrap every tree sees all N rows and the trees differ
  only through their tree ids;
* draw i of tree b takes Philox4x32-10 word (i mod 4) of the counter
  (i div 4, BOOT_STREAM, 0xFFFFFFFF, tree0 + b) under the seed key and maps
  the word w to row floor(w * N / 2^32);
* classification: every tree votes for its leaf's majority class (smallest
  class id on ties) and the forest predicts the class with most votes
  (smallest class id on ties); regression: the mean of the trees' leaf means,
  summed in tree order.

Boost (gradient boosting with shrinkage lr, one round after another)
* regression: F_0 = mean(y); round m fits an SLR tree (MSE criterion) with
  tree id tree0 + m to the residuals y - F_{m-1} and adds lr times its leaf
  mean: F_m = F_{m-1} + lr * h_m(x);
* classification (K classes, softmax): F_0 = 0; round m computes
  p = softmax(F_{m-1}) and, for every class k, fits an SLR tree with tree id
  tree0 + m * K + k to the pseudo-residuals 1{y = k} - p_k (the negative
  gradient of the multinomial log-loss) and adds lr times its leaf mean to
  F_k; the prediction is the argmax of F (smallest class on ties);
* a leaf's value is the plain mean of its residuals (first-order step; no
  Newton leaf weights or regularisation).

Routing for prediction is oracle.tree's: right iff float32(a^T x) >= t.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import split as S
from . import tree as T
from .philox import philox4x32_10, seed_key

BOOT_STREAM = 0x80000000      # word 1 of every bootstrap draw
NO_NODE = 0xFFFFFFFF          # word 2: a draw that belongs to no node


def bootstrap_indices(seed: int, tree: int, N: int):
    """N row indices drawn with replacement for tree id `tree` (int64 [N])."""
    if N <= 0:
        return np.zeros(0, dtype=np.int64)
    groups = (N + 3) // 4
    ctr = np.zeros((groups, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(groups, dtype=np.uint64)
    ctr[:, 1] = BOOT_STREAM
    ctr[:, 2] = NO_NODE
    ctr[:, 3] = tree & 0xFFFFFFFF
    words = philox4x32_10(ctr, seed_key(seed)).reshape(-1)[:N].astype(np.uint64)
    return ((words * np.uint64(N)) >> np.uint64(32)).astype(np.int64)


@dataclasses.dataclass
class Forest:
    trees: list
    samples: list          # row indices each tree was grown on
    K: int


def grow_forest(X, target, prm: T.TreeParams, n_trees: int, bootstrap: bool = True):
    """B SLM trees, tree b on bootstrap sample b (or on all rows)."""
    X = np.asarray(X)
    target = np.asarray(target)
    N = X.shape[0]
    trees, samples = [], []
    for b in range(n_trees):
        tid = prm.tree + b
        idx = bootstrap_indices(prm.seed, tid, N) if bootstrap else np.arange(N)
        p = dataclasses.replace(prm, tree=tid)
        trees.append(T.grow_tree(X[idx], target[idx], p))
        samples.append(idx)
    return Forest(trees=trees, samples=samples, K=prm.K if prm.crit != S.MSE else 0)


def tree_outputs(forest: Forest, X):
    """[B, n] per-tree predictions: class ids, or leaf means for regression."""
    return np.stack([T.predict(t, X) for t in forest.trees])


def combine(outputs, K: int):
    """Forest output from the per-tree outputs [B, n]: majority vote over class
    ids (smallest class on ties) when K > 0, else the mean in tree order."""
    outputs = np.asarray(outputs)
    if K > 0:
        votes = np.zeros((outputs.shape[1], K), dtype=np.int64)
        for b in range(outputs.shape[0]):
            votes[np.arange(outputs.shape[1]), outputs[b].astype(np.int64)] += 1
        return np.argmax(votes, axis=1)
    acc = np.zeros(outputs.shape[1], dtype=np.float64)
    for b in range(outputs.shape[0]):
        acc = acc + outputs[b]
    return acc / outputs.shape[0]


def forest_predict(forest: Forest, X):
    return combine(tree_outputs(forest, X), forest.K)


# ---------------------------------------------------------------- boosting
@dataclasses.dataclass
class Boost:
    F0: np.ndarray          # [max(K, 1)] initial score(s)
    trees: list             # round-major: rounds x max(K, 1) trees
    lr: float
    K: int


def leaf_values(tr: T.Tree, X):
    """h(x): the leaf mean reached by every row (regression trees)."""
    return T.predict(tr, X)


def softmax(F):
    m = F.max(axis=1, keepdims=True)
    e = np.exp(F - m)
    return e / e.sum(axis=1, keepdims=True)


def _mse_params(prm: T.TreeParams, tid: int):
    return dataclasses.replace(prm, crit=S.MSE, K=0, tree=tid)


def boost_regression(X, y, prm: T.TreeParams, n_rounds: int, lr: float):
    """SLR Boost: returns (model, F after every round [n_rounds + 1, N])."""
    X = np.asarray(X)
    y = np.asarray(y, dtype=np.float64)
    F = np.full(y.shape, S.exact_sum(y) / y.size)
    hist = [F.copy()]
    trees = []
    for m in range(n_rounds):
        tr = T.grow_tree(X, y - F, _mse_params(prm, prm.tree + m))
        trees.append(tr)
        F = F + lr * leaf_values(tr, X)
        hist.append(F.copy())
    return Boost(F0=np.array([hist[0][0]]), trees=trees, lr=lr, K=0), np.stack(hist)


def boost_classification(X, y, K: int, prm: T.TreeParams, n_rounds: int, lr: float):
    """SLM Boost (K-class softmax): returns (model, F after every round
    [n_rounds + 1, N, K])."""
    X = np.asarray(X)
    y = np.asarray(y, dtype=np.int64)
    F = np.zeros((y.size, K))
    onehot = np.eye(K)[y]
    hist = [F.copy()]
    trees = []
    for m in range(n_rounds):
        R = onehot - softmax(F)
        step = np.zeros_like(F)
        for k in range(K):
            tr = T.grow_tree(X, R[:, k], _mse_params(prm, prm.tree + m * K + k))
            trees.append(tr)
            step[:, k] = leaf_values(tr, X)
        F = F + lr * step
        hist.append(F.copy())
    return Boost(F0=np.zeros(K), trees=trees, lr=lr, K=K), np.stack(hist)


def boost_scores(model: Boost, X):
    """F(x) of a boosted model: [n] (regression) or [n, K]."""
    X = np.asarray(X)
    Kc = max(model.K, 1)
    F = np.tile(model.F0, (X.shape[0], 1)).astype(np.float64)
    for i, tr in enumerate(model.trees):
        F[:, i % Kc] += model.lr * leaf_values(tr, X)
    return F if model.K > 0 else F[:, 0]


def boost_predict(model: Boost, X):
    F = boost_scores(model, X)
    return np.argmax(F, axis=1) if model.K > 0 else F
