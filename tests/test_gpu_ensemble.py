"""GPU forest and boosting (slm_grow_forest, slm_forest_predict, slm_boost)
against the oracle (oracle.ensemble):

* bootstrap draws bit-exact with the oracle's, and the gathered targets (the
  roots' class counts) exact;
* every tree of a forest grown together equals the tree slm_grow_tree grows
  alone on that tree's sample with that tree id;
* forest prediction: leaves bit-exact with the float32 routing rule, votes /
  means bit-exact with the oracle's combination of the per-tree outputs;
* held-out accuracy / MSE of the GPU forest close to the oracle forest's;
* boosting: the initial scores, every round's residual targets (the roots'
  means), the score update (bit-exact from the trees), a falling training
  loss, and training loss close to the oracle's.
"""
import numpy as np
import pytest
import torch

from oracle import ensemble as E
from oracle import split as OS
from oracle import tree as OT
from paper_2208_07023_amd import inputs

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _route(tr, X, root=0):
    """Leaf of every row: right iff float32 dot (FP32 sums in dimension order)
    >= thr, starting at `root` (global indices)."""
    node = np.full(X.shape[0], root, dtype=np.int64)
    for _ in range(64):
        internal = tr["left"][node] >= 0
        if not internal.any():
            break
        z = np.zeros(X.shape[0], np.float32)
        for d in range(X.shape[1]):
            z = (z + (tr["w"][node, d] * X[:, d]).astype(np.float32)).astype(np.float32)
        nxt = np.where(z >= tr["thr"][node], tr["right"][node], tr["left"][node])
        node = np.where(internal, nxt, node)
    return node


def _oracle_params(cfg):
    return OT.TreeParams(crit=cfg.crit, K=cfg.K, max_depth=cfg.max_depth, min_node=cfg.min_node,
                         P=cfg.P, T=cfg.T, bins=cfg.bins, omega=cfg.omega, c1=cfg.c1, c2=cfg.c2,
                         seed=cfg.seed, tree=cfg.tree)


@pytest.mark.parametrize("N,n_trees", [(1003, 3), (1, 2), (4096, 5)])
def test_bootstrap_samples_match_oracle(gpu_lib, N, n_trees):
    api = gpu_lib
    X, y = inputs.cluster_mixture(N, 6, 3, seed=N)
    cfg = api.TreeConfig(crit=api.GINI, K=3, max_depth=0, P=8, T=1, bins=16, seed=77, tree=5)
    f = api.grow_forest(_t(X), _t(y), cfg, n_trees, return_samples=True)
    S = f["samples"].cpu().numpy()
    assert f["n_nodes"] == n_trees and np.array_equal(f["tree_of"], np.arange(n_trees))
    for b in range(n_trees):
        ref = E.bootstrap_indices(77, 5 + b, N)
        assert np.array_equal(S[b], ref), b
        assert np.array_equal(f["leaf"][b], np.bincount(y[ref], minlength=3)), b
        assert f["n"][b] == N


def test_regression_bootstrap_gathers_targets(gpu_lib):
    api = gpu_lib
    X, y = inputs.friedman1(2001, 7, seed=3)
    cfg = api.TreeConfig(crit=api.MSE, K=0, max_depth=0, P=8, T=1, bins=16, seed=4)
    f = api.grow_forest(_t(X), _t(y), cfg, 3, return_samples=True)
    for b in range(3):
        idx = E.bootstrap_indices(4, b, 2001)
        assert np.array_equal(f["samples"][b].cpu().numpy(), idx)
        assert f["leaf"][b][0] == pytest.approx(y[idx].mean(), rel=1e-12)


@pytest.mark.parametrize("crit,bins,bootstrap", [(0, 64, True), (1, 256, True), (0, 0, False)])
def test_forest_trees_equal_trees_grown_alone(gpu_lib, crit, bins, bootstrap):
    api = gpu_lib
    N, D, K, nt = 6000, 10, 3, 3
    X, y = inputs.cluster_mixture(N, D, K, clusters_per_class=2, seed=11)
    cfg = api.TreeConfig(crit=crit, K=K, max_depth=4, min_node=16, P=32, T=6, bins=bins, seed=3,
                         tree=20)
    f = api.grow_forest(_t(X), _t(y), cfg, nt, bootstrap=bootstrap)
    assert np.array_equal(f["tree_of"][:nt], np.arange(nt))
    for b in range(nt):
        idx = E.bootstrap_indices(3, 20 + b, N) if bootstrap else np.arange(N)
        cfg.tree = 20 + b
        alone = api.grow_tree(_t(X[idx]), _t(y[idx]), cfg)
        cfg.tree = 20
        mine = api.forest_tree(f, b)
        assert mine["n_nodes"] == alone["n_nodes"], b
        for k in ("w", "thr", "left", "right", "leaf", "n", "split_loss", "heap", "depth"):
            assert np.array_equal(mine[k], alone[k]), (b, k)
    # and a graph replay of the forest reproduces it
    cfg.use_graph = True
    g = api.grow_forest(_t(X), _t(y), cfg, nt, bootstrap=bootstrap)
    for k in ("w", "thr", "left", "right", "tree_of"):
        assert np.array_equal(f[k], g[k]), k


@pytest.mark.parametrize("crit,K", [(OS.ENTROPY, 4), (OS.MSE, 0)])
def test_forest_predict_matches_oracle_combination(gpu_lib, crit, K):
    api = gpu_lib
    D, nt = 9, 5
    if crit == OS.MSE:
        X, y = inputs.friedman1(5000, D, seed=5)
        Xt, _ = inputs.friedman1(3001, D, seed=6)
    else:
        X, y = inputs.cluster_mixture(5000, D, K, seed=5)
        Xt, _ = inputs.cluster_mixture(3001, D, K, seed=6)
    cfg = api.TreeConfig(crit=crit, K=K, max_depth=5, min_node=8, P=32, T=5, bins=64, seed=8)
    f = api.grow_forest(_t(X), _t(y), cfg, nt)
    out, leaves = api.forest_predict(f, _t(Xt), return_leaves=True)
    out, leaves = out.cpu().numpy(), leaves.cpu().numpy()
    per_tree = []
    for b in range(nt):
        lf = _route(f, Xt, root=b)
        assert np.array_equal(leaves[b], lf), b
        assert np.all(f["tree_of"][lf] == b)
        per_tree.append(np.argmax(f["leaf"][lf], axis=1) if K else f["leaf"][lf, 0])
    ref = E.combine(np.stack(per_tree), K)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("crit,K", [(OS.GINI, 3), (OS.MSE, 0)])
def test_forest_quality_close_to_oracle(gpu_lib, crit, K):
    api = gpu_lib
    D, nt = 6, 4
    # 20 000 training and 20 000 held-out rows
    if crit == OS.MSE:
        X, y = inputs.friedman1(20000, D, noise=0.5, seed=12)
        Xt, yt = inputs.friedman1(20000, D, noise=0.5, seed=13)
    else:
        # one distribution (the cluster means are drawn from the seed), split
        Xa, ya = inputs.cluster_mixture(40000, D, K, mean_std=1.0, seed=12)
        X, y, Xt, yt = Xa[:20000], ya[:20000], Xa[20000:], ya[20000:]
    cfg = api.TreeConfig(crit=crit, K=K, max_depth=4, min_node=16, P=16, T=5, bins=32, seed=2)
    g = api.grow_forest(_t(X), _t(y), cfg, nt)
    pg = api.forest_predict(g, _t(Xt)).cpu().numpy()
    o = E.grow_forest(X, y, _oracle_params(cfg), nt)
    po = E.forest_predict(o, Xt)
    if K:
        acc_g, acc_o = (pg == yt).mean(), (po == yt).mean()
        print(f"forest held-out accuracy gpu {acc_g:.4f} oracle {acc_o:.4f}")
        assert abs(acc_g - acc_o) <= 0.005 + 1e-12
    else:
        mse_g, mse_o = ((pg - yt) ** 2).mean(), ((po - yt) ** 2).mean()
        print(f"forest held-out MSE gpu {mse_g:.4f} oracle {mse_o:.4f}")
        assert mse_g <= 1.03 * mse_o
        # the mean aggregate never does worse than the mean tree, pointwise
        outs = np.stack([api.predict(api.forest_tree(g, b), _t(Xt)) for b in range(nt)])
        assert np.all((pg - yt) ** 2 <= ((outs - yt) ** 2).mean(axis=0) + 1e-9)


def _softmax(F):
    m = F.max(axis=1, keepdims=True)
    e = np.exp(F - m)
    return e / e.sum(axis=1, keepdims=True)


@pytest.mark.parametrize("n_classes", [0, 3])
def test_boost_rounds_follow_the_gradient_steps(gpu_lib, n_classes):
    api = gpu_lib
    N, D, lr, M = 3000, 8, 0.3, 3
    if n_classes:
        X, y = inputs.cluster_mixture(N, D, n_classes, seed=21)
    else:
        X, y = inputs.friedman1(N, D, seed=21)
    cfg = api.TreeConfig(crit=api.MSE, K=0, max_depth=3, min_node=16, P=16, T=4, bins=64, seed=6,
                         tree=2)
    Xd = _t(X)
    m = api.boost(Xd, _t(y), cfg, M, lr, n_classes=n_classes)
    Kc = max(1, n_classes)
    onehot = np.eye(Kc)[y] if n_classes else None
    # initial scores
    if n_classes:
        assert np.array_equal(m["F0"], np.zeros(Kc))
    else:
        assert m["F0"][0] == pytest.approx(y.mean(), rel=1e-12)
    # scores after every round, from the trees (bit-exact at the end)
    Fs = [api.boost_scores(m, Xd, rounds=r).cpu().numpy() for r in range(M + 1)]
    assert np.array_equal(Fs[-1], m["F"].cpu().numpy())
    assert np.array_equal(Fs[0], np.tile(m["F0"], (N, 1)))
    roots = [int(np.nonzero(m["tree_of"] == t)[0][0]) for t in range(M * Kc)]
    losses = []
    for r in range(M):
        F = Fs[r]
        R = onehot - _softmax(F) if n_classes else (y - F[:, 0])[:, None]
        for k in range(Kc):
            root = roots[r * Kc + k]
            # the tree was grown on the residuals of the scores before its round
            assert m["n"][root] == N
            assert m["leaf"][root][0] == pytest.approx(R[:, k].mean(), rel=1e-9, abs=1e-12)
            # and its leaf values, routed by the prediction rule, are the step
            lf = _route(m, X, root=root)
            step = lr * m["leaf"][lf, 0]
            assert np.array_equal(Fs[r + 1][:, k], F[:, k] + step)
        if n_classes:
            losses.append(-np.mean(np.log(_softmax(F)[np.arange(N), y])))
        else:
            losses.append(np.mean((y - F[:, 0]) ** 2))
    final = (-np.mean(np.log(_softmax(Fs[-1])[np.arange(N), y])) if n_classes
             else np.mean((y - Fs[-1][:, 0]) ** 2))
    losses.append(final)
    print("training loss by round", np.round(losses, 5))
    assert all(b < a for a, b in zip(losses, losses[1:])), losses


@pytest.mark.parametrize("n_classes", [0, 3])
def test_boost_training_loss_close_to_oracle(gpu_lib, n_classes):
    api = gpu_lib
    N, D, lr, M = 1200, 6, 0.5, 3
    if n_classes:
        X, y = inputs.cluster_mixture(N, D, n_classes, seed=31)
    else:
        X, y = inputs.friedman1(N, D, noise=0.5, seed=31)
    cfg = api.TreeConfig(crit=api.MSE, K=0, max_depth=3, min_node=16, P=16, T=5, bins=32, seed=1)
    g = api.boost(_t(X), _t(y), cfg, M, lr, n_classes=n_classes)
    Fg = g["F"].cpu().numpy()
    prm = _oracle_params(cfg)
    if n_classes:
        _, Fo = E.boost_classification(X, y, n_classes, prm, M, lr)
        lg = -np.mean(np.log(_softmax(Fg)[np.arange(N), y]))
        lo = -np.mean(np.log(_softmax(Fo[-1])[np.arange(N), y]))
    else:
        _, Fo = E.boost_regression(X, y, prm, M, lr)
        lg = np.mean((y - Fg[:, 0]) ** 2)
        lo = np.mean((y - Fo[-1]) ** 2)
    print(f"boost training loss gpu {lg:.5f} oracle {lo:.5f}")
    assert lg <= 1.05 * lo


def test_bf16_forest_with_odd_rows_equals_trees_alone(gpu_lib):
    """Screened (bfloat16 X) forest with D odd: 26-byte rows take the gather's
    2-byte path; every tree still equals the tree grown alone."""
    from oracle import screen as SC
    api = gpu_lib
    N, D, K, nt = 5000, 13, 3, 2
    X, y = inputs.cluster_mixture(N, D, K, seed=31)
    X = SC.bf16_round(X)
    Xb = torch.from_numpy(X).cuda().to(torch.bfloat16)
    cfg = api.TreeConfig(crit=api.GINI, K=K, max_depth=3, min_node=16, P=32, T=4, bins=64, seed=9,
                         precision=1, rescore_k=8, tree=4)
    f = api.grow_forest(Xb, _t(y), cfg, nt, return_samples=True)
    for b in range(nt):
        idx = E.bootstrap_indices(9, 4 + b, N)
        assert np.array_equal(f["samples"][b].cpu().numpy(), idx)
        cfg.tree = 4 + b
        alone = api.grow_tree(Xb[torch.from_numpy(idx).cuda()].contiguous(), _t(y[idx]), cfg)
        cfg.tree = 4
        mine = api.forest_tree(f, b)
        for k in ("w", "thr", "left", "right", "n", "split_loss"):
            assert np.array_equal(mine[k], alone[k]), (b, k)


def test_many_trees_scan_what_they_partition(gpu_lib):
    """Twelve trees grown together over 96 000 stacked rows: the deeper
    depths search a sparse subset of the rows (nodes of other trees stopped),
    spread over several chunks each.  Every split's histogram loss equals the
    size-weighted impurity of the children the partition made (the scan
    binned exactly the node's rows), the children's class counts add up to
    the parent's, and each tree equals the one grown alone."""
    api = gpu_lib
    N, D, K, nt = 8000, 12, 3, 12
    X, y = inputs.cluster_mixture(N, D, K, clusters_per_class=3, seed=21)
    cfg = api.TreeConfig(crit=OS.ENTROPY, K=K, max_depth=6, min_node=64, P=64, T=4, bins=128,
                         seed=7, tree=40, use_graph=True)
    f = api.grow_forest(_t(X), _t(y), cfg, nt)
    depths = set()
    for b in range(nt):
        tr = api.forest_tree(f, b)
        n = tr["n"]
        for i in range(tr["n_nodes"]):
            l, r = tr["left"][i], tr["right"][i]
            if l < 0:
                continue
            depths.add(int(tr["depth"][i]))
            assert n[l] + n[r] == n[i] and n[l] > 0 and n[r] > 0
            w = (n[l] * tr["impurity"][l] + n[r] * tr["impurity"][r]) / n[i]
            assert w == pytest.approx(tr["split_loss"][i], rel=1e-9, abs=1e-12), (b, i)
            assert np.array_equal(tr["leaf"][l] + tr["leaf"][r], tr["leaf"][i]), (b, i)
        if b % 4 == 0:
            idx = E.bootstrap_indices(7, 40 + b, N)
            cfg.tree = 40 + b
            alone = api.grow_tree(_t(X[idx]), _t(y[idx]), cfg)
            cfg.tree = 40
            assert tr["n_nodes"] == alone["n_nodes"], b
            for k in ("w", "thr", "left", "right", "leaf", "n", "split_loss"):
                assert np.array_equal(tr[k], alone[k]), (b, k)
    assert len(depths) >= 3
