"""Oracle: SLM tree built on the swarm's global-best split (Sec. III-B, Alg. 2)
and tree prediction (Sec. II-A, Eqs. (3)-(4)).

Readings of the paper used here:
* a node is split when it is deep enough to allow it (depth < max_depth), holds
  at least min_node samples and is impure (classification: impurity > 0;
  regression: not all targets equal) -- the paper's "pure enough" and "small
  enough" stopping rule (Sec. II-A);
* search = 2 replaces the swarm by the probabilistic search over the node's
  top ps_R DFT channels (oracle.probsearch); search = 1 runs the adaptive
  swarm (oracle.apso) instead of the plain one;
* the swarm runs in all D input dimensions unless dft_top_n = n with
  0 < n < D: then every searched node first runs the DFT and the swarm
  starts in the span of its top n channels (oracle.dft; Alg. 2);
* the split is kept only if the global-best loss is strictly below the node's
  own impurity; the children are the samples with a^T x >= t (right) and
  a^T x < t (left), in their original order;
* leaves predict the majority class (smallest class id on ties) or, for
  regression, the mean target;
* nodes are visited breadth first, left child before right; a node's swarm
  is keyed by its heap id (root 0, children 2j+1 and 2j+2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import apso
from . import dft
from . import probsearch
from . import screen
from . import split as S
from .pso import run_pso


@dataclass
class TreeParams:
    crit: int = S.ENTROPY
    K: int = 2
    max_depth: int = 8
    min_node: int = 32
    P: int = 32
    T: int = 20
    bins: int = 256            # 0 = exact scan
    omega: float = 0.7
    c1: float = 1.5
    c2: float = 1.5
    seed: int = 0
    tree: int = 0
    precision: int = 0         # 1 = bfloat16 screening, float32 re-scoring
    rescore_k: int = 32
    dft_top_n: int = 0         # 0 < n < D: swarm in the node's top n DFT channels
    search: int = 0            # 0 = swarm (Alg. 1); 1 = APSO (Sec. III-B); 2 = probabilistic
                               # search (Sec. II-B)
    ps_R: int = 8              # probabilistic search: ranks combined
    ps_alpha0: float = 10.0    # probabilistic search: coefficient range of rank 1


@dataclass
class Tree:
    D: int
    K: int
    w: list = field(default_factory=list)         # float32 [D] per node
    thr: list = field(default_factory=list)
    left: list = field(default_factory=list)
    right: list = field(default_factory=list)
    leaf: list = field(default_factory=list)      # class counts [K] or [mean]
    heap: list = field(default_factory=list)
    depth: list = field(default_factory=list)
    n: list = field(default_factory=list)
    impurity: list = field(default_factory=list)
    split_loss: list = field(default_factory=list)
    rows: list = field(default_factory=list)      # sample indices per node

    def arrays(self):
        nn = len(self.thr)
        return dict(w=np.array(self.w, dtype=np.float32).reshape(nn, self.D),
                    thr=np.array(self.thr, dtype=np.float32),
                    left=np.array(self.left, dtype=np.int64),
                    right=np.array(self.right, dtype=np.int64),
                    leaf=np.array(self.leaf, dtype=np.float64),
                    heap=np.array(self.heap, dtype=np.int64),
                    depth=np.array(self.depth, dtype=np.int64),
                    n=np.array(self.n, dtype=np.int64),
                    impurity=np.array(self.impurity),
                    split_loss=np.array(self.split_loss))


def node_summary(target, crit, K):
    """(impurity, splittable-by-purity, leaf value) of one node's targets."""
    if crit == S.MSE:
        y = np.asarray(target, dtype=np.float64)
        imp = S.mse_node(y)
        impure = y.size > 0 and y.max() > y.min()
        mean = S.exact_sum(y) / y.size if y.size else 0.0
        return imp, impure, [mean]
    c = np.bincount(np.asarray(target, dtype=np.int64), minlength=K)[:K]
    imp = S.gini_node(c) if crit == S.GINI else S.entropy_node(c)
    return imp, imp > 0, c.astype(np.float64).tolist()


def evaluate_node(Xn, tn, prm: TreeParams):
    """Evaluation closure for run_pso: project the node's rows on the float32
    directions, round the FP64 projections to float32 and scan each column.
    With precision = 1 the evaluation is the screened one of oracle.screen
    (X then holds bfloat16 values)."""
    if prm.precision == 1:
        return screen.evaluate_screened(Xn, tn, prm.crit, prm.K, prm.bins, prm.rescore_k)

    def ev(W32):
        Z = S.project(Xn, W32).astype(np.float32)
        loss = np.empty(W32.shape[0])
        spl = np.empty(W32.shape[0], dtype=np.int64)
        thr = np.empty(W32.shape[0], dtype=np.float32)
        for p in range(W32.shape[0]):
            r = (S.scan_exact(Z[:, p], tn, prm.crit, prm.K) if prm.bins == 0
                 else S.scan_hist(Z[:, p], tn, prm.bins, prm.crit, prm.K))
            loss[p], spl[p], thr[p] = r["loss"], r["split"], r["thr"]
        return loss, spl, thr
    return ev


def grow_tree(X, target, prm: TreeParams, rows=None, keep_rows=False):
    """Alg. 2 applied breadth first from the root; returns a Tree."""
    X = np.asarray(X)
    D = X.shape[1]
    target = np.asarray(target)
    tr = Tree(D=D, K=prm.K)
    root_rows = np.arange(X.shape[0]) if rows is None else np.asarray(rows)
    frontier = [(root_rows, 0, 0)]           # (rows, heap id, depth)
    while frontier:
        nxt = []
        for rws, hid, dep in frontier:
            idx = len(tr.thr)
            imp, impure, leafv = node_summary(target[rws], prm.crit, prm.K)
            tr.w.append(np.zeros(D, dtype=np.float32))
            tr.thr.append(np.float32(np.inf))
            tr.left.append(-1)
            tr.right.append(-1)
            tr.leaf.append(leafv)
            tr.heap.append(hid)
            tr.depth.append(dep)
            tr.n.append(len(rws))
            tr.impurity.append(imp)
            tr.split_loss.append(np.inf)
            if keep_rows:
                tr.rows.append(rws)
            if not (dep < prm.max_depth and len(rws) >= prm.min_node and impure):
                continue
            Xn = X[rws]
            tn = target[rws]
            x0 = None
            if prm.search == 2:
                R = min(prm.ps_R, D)
                ranks = dft.top_n(dft.dft_losses(Xn, tn, prm.crit, prm.K, prm.bins), R)
                pd, am = probsearch.tables(R, prm.ps_alpha0)
                res = probsearch.run_search(evaluate_node(Xn, tn, prm), prm.P, D, prm.T, prm.seed,
                                            prm.tree, hid, ranks, pd, am)
            sel = None
            if prm.search != 2 and 0 < prm.dft_top_n < D:
                sel = dft.top_n(dft.dft_losses(Xn, tn, prm.crit, prm.K, prm.bins), prm.dft_top_n)
                x0 = dft.subspace_start(prm.seed, prm.tree, hid, prm.P, D, sel)
            if prm.search == 1:
                res = apso.run_apso(evaluate_node(Xn, tn, prm), prm.P, D, prm.T, prm.seed,
                                    prm.tree, hid, x0=x0, dims=sel)
            elif prm.search != 2:
                res = run_pso(evaluate_node(Xn, tn, prm), prm.P, D, prm.T, prm.omega,
                              prm.c1, prm.c2, prm.seed, prm.tree, hid, x0=x0)
            tr.split_loss[idx] = res["loss"]
            if not res["loss"] < imp:
                continue
            w32 = res["gbest"].astype(np.float32)
            z = S.project(Xn, w32[None, :])[:, 0].astype(np.float32)
            right = z >= res["thr"]
            tr.w[idx] = w32
            tr.thr[idx] = np.float32(res["thr"])
            nxt.append((idx, rws[~right], 2 * hid + 1, dep + 1))
            nxt.append((idx, rws[right], 2 * hid + 2, dep + 1))
        frontier = []
        for k, (parent, rws, hid, dep) in enumerate(nxt):
            child = len(tr.thr) + k
            if hid == 2 * tr.heap[parent] + 1:
                tr.left[parent] = child
            else:
                tr.right[parent] = child
            frontier.append((rws, hid, dep))
    return tr


def predict(tr: Tree, X):
    """Route each sample from the root: right iff float32(a^T x) >= t, with the
    projection formed the same way as in the partition above.
    Returns class ids (classification) or means (regression)."""
    A = tr.arrays()
    X = np.asarray(X)
    Zall = S.project(X, A["w"]).astype(np.float32)      # [n_samples, n_nodes]
    node = np.zeros(X.shape[0], dtype=np.int64)
    for _ in range(int(A["depth"].max()) + 1):
        internal = A["left"][node] >= 0
        if not internal.any():
            break
        ii = np.nonzero(internal)[0]
        nd = node[ii]
        go_right = Zall[ii, nd] >= A["thr"][nd]
        node[ii] = np.where(go_right, A["right"][nd], A["left"][nd])
    leaf = A["leaf"][node]
    if tr.K > 1:
        return np.argmax(leaf, axis=1)
    return leaf[:, 0]
