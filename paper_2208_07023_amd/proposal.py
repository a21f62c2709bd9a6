"""Learned proposal: harvesting training pairs, training the network and
comparing learned against random swarm starts, all on the GPU through the C
ABI (node statistics, network forward/backward, loss, Adam and the node-batch
search run in this library's kernels; torch holds the tensors, draws the
minibatch order and moves rows).

Pairs are (node statistics, standardised global-best direction) of every node
that plain-PSO trees split, on seeded class mixtures.  The network maps the
statistics to M seeds; a learned start places the first M particles of a
swarm on them, and the swarm runs unchanged -- its loss remains the judge, and
the comparison below runs both starts to the same loss target.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import api, inputs


@dataclass
class Net:
    params: torch.Tensor      # packed float32 parameters on the device
    n_in: int
    hidden: int
    n_out: int
    n_seeds: int
    D: int
    K: int


def init_params(n_in: int, hidden: int, n_out: int, seed: int, device="cuda") -> torch.Tensor:
    """Weights ~ N(0, 1/fan_in) (the last layer scaled by 1/4), biases 0;
    drawn with numpy's PCG64 and copied to the device."""
    rng = np.random.default_rng(seed)
    parts = []
    shapes = [(hidden, n_in), (hidden,), (hidden, hidden), (hidden,), (n_out, hidden), (n_out,)]
    for i, shp in enumerate(shapes):
        if len(shp) == 1:
            parts.append(np.zeros(shp[0]))
        else:
            sc = 1.0 / math.sqrt(shp[1]) * (0.25 if i == 4 else 1.0)
            parts.append((rng.standard_normal(shp) * sc).ravel())
    return torch.from_numpy(np.concatenate(parts).astype(np.float32)).to(device)


# ------------------------------------------------------------------ harvesting
def cluster_mixture_gpu(n: int, d: int, k: int, clusters_per_class: int, mean_std: float,
                        seed: int, device="cuda"):
    """The class-mixture recipe of inputs.cluster_mixture (cluster means
    ~N(0, mean_std^2 I), per-dimension variances ~U[0.5, 2], balanced labels),
    drawn with torch's device generator so large harvests do not wait on the
    host.  Returns (X float32 [n, d], y int32 [n]) on the device."""
    g = torch.Generator(device=device).manual_seed(seed)
    c = clusters_per_class
    means = torch.randn(k, c, d, generator=g, device=device) * mean_std
    var = torch.rand(k, c, d, generator=g, device=device) * 1.5 + 0.5
    y = (torch.arange(n, device=device) % k)[torch.randperm(n, generator=g, device=device)]
    cl = torch.randint(0, c, (n,), generator=g, device=device)
    X = means[y, cl] + torch.randn(n, d, generator=g, device=device) * var[y, cl].sqrt()
    return X.float().contiguous(), y.to(torch.int32).contiguous()


def harvest(n_trees: int, D: int, K: int, n_lo: int, n_hi: int, seed: int, P: int = 64,
            T: int = 50, max_depth: int = 8, mean_std=(0.4, 1.5), clusters: int = 4,
            device="cuda", log=None):
    """Grow plain-PSO trees on seeded class mixtures (K classes x `clusters`
    clusters, N log-uniform in [n_lo, n_hi], cluster spread uniform in mean_std) and
    return the pairs of every split node: stats [n, (K+1) D], sigma [n, D],
    targets [n, D] (device float32)."""
    rng = np.random.default_rng(seed)
    S, G, W = [], [], []
    for t in range(n_trees):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        ms = float(rng.uniform(*mean_std))
        X, y = cluster_mixture_gpu(n, D, K, clusters, ms, int(rng.integers(1 << 31)), device)
        cfg = api.TreeConfig(crit=api.ENTROPY, K=K, max_depth=max_depth, min_node=32, P=P, T=T,
                             bins=256, seed=seed, tree=t)
        tr = api.grow_tree(X, y, cfg, stats=True)
        split = tr["left"] >= 0
        S.append(tr["stats"][split])
        G.append(tr["sigma"][split])
        W.append(tr["w"][split])
        if log and (t + 1) % max(1, n_trees // 10) == 0:
            log(f"harvest: {t + 1}/{n_trees} trees, {sum(len(s) for s in S)} pairs")
    stats = torch.from_numpy(np.concatenate(S)).to(device)
    sigma = torch.from_numpy(np.concatenate(G)).to(device)
    w = torch.from_numpy(np.concatenate(W)).to(device)
    w = w.contiguous()
    return stats, sigma, api.proposal_targets(w, sigma)


# ------------------------------------------------------------------ training
def train(stats, targets, D: int, K: int, n_seeds: int = 64, hidden: int = 256, epochs: int = 20,
          batch: int = 4096, lr: float = 1e-3, eps: float = 0.05, seed: int = 0, log=None):
    """Adam on the relaxed winner-take-all loss; returns (Net, loss history
    per epoch)."""
    n_in, n_out = (K + 1) * D, n_seeds * D
    dev = stats.device
    params = init_params(n_in, hidden, n_out, seed, dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    n = stats.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    step = 0
    for ep in range(epochs):
        order = torch.randperm(n, generator=gen).to(dev)
        tot, cnt = 0.0, 0
        for b0 in range(0, n, batch):
            idx = order[b0:b0 + batch]
            sb = stats.index_select(0, idx).contiguous()
            tb = targets.index_select(0, idx).contiguous()
            B = sb.shape[0]
            out, cache = api.mlp_forward(params, n_in, hidden, n_out, sb)
            loss, d_out = api.wta_loss(out, tb, n_seeds, eps, scale=1.0 / B)
            grads = api.mlp_backward(params, n_in, hidden, n_out, sb, cache, d_out)
            step += 1
            api.adam_step(params, grads, m, v, lr=lr, step=step)
            tot += float(loss.sum())
            cnt += B
        hist.append(tot / max(1, cnt))
        if log:
            log(f"train: epoch {ep + 1}/{epochs} loss {hist[-1]:.4f}")
    return Net(params, n_in, hidden, n_out, n_seeds, D, K), hist


def mean_best_cos2(net: Net, stats, targets, bf16: bool = True) -> float:
    """Mean over pairs of max_i (u_i . t)^2 (1 = a seed on the target's line),
    from the relaxed loss with eps = 0."""
    out, _ = api.mlp_forward(net.params, net.n_in, net.hidden, net.n_out, stats, bf16=bf16)
    loss, _ = api.wta_loss(out, targets, net.n_seeds, 0.0)
    return float(1.0 - loss.mean())


# ------------------------------------------------------------------ comparison
def _route_depths(tr, X):
    """Rows of every searched node of a grown tree, by depth: list of
    (node indices, row index arrays).  Routing follows the tree's stored
    float32 rule (right iff float32(w.x) >= t) on the host."""
    n_nodes = tr["n_nodes"]
    rows = {0: np.arange(X.shape[0])}
    by_depth = {}
    for i in range(n_nodes):
        r = rows.get(i)
        if r is None:
            continue
        if np.isfinite(tr["split_loss"][i]):
            by_depth.setdefault(int(tr["depth"][i]), []).append((i, r))
        if tr["left"][i] >= 0:
            z = (X[r].astype(np.float64) @ tr["w"][i].astype(np.float64)).astype(np.float32)
            right = z >= tr["thr"][i]
            rows[int(tr["left"][i])] = r[~right]
            rows[int(tr["right"][i])] = r[right]
    return [by_depth[d] for d in sorted(by_depth)]


def compare_starts(net: Net, X, y, K: int, ref_P: int = 256, ref_T: int = 200, P: int = 64,
                   T_max: int = 50, tol: float = 0.01, max_depth: int = 8, seed: int = 0,
                   tree: int = 0, device="cuda", log=None):
    """Paired comparison of random and learned swarm starts on one tree.

    A reference tree grown with plain PSO at an extended budget (ref_P
    particles, ref_T moves) fixes the node row sets and each node's reference
    loss L_ref.  On exactly those nodes, batched per depth, each arm searches
    with P particles until its global-best loss is <= (1 + tol) L_ref or after
    T_max moves.  Returns per-arm totals: wall ms (including the learned arm's
    statistics and inference), evaluations, nodes that met the target."""
    Xd = torch.from_numpy(X).to(device)
    yd = torch.from_numpy(y).to(device)
    ref_cfg = api.TreeConfig(crit=api.ENTROPY, K=K, max_depth=max_depth, min_node=32, P=ref_P,
                             T=ref_T, bins=256, seed=seed + 1, tree=tree)
    ref = api.grow_tree(Xd, yd, ref_cfg)
    depths = _route_depths(ref, X)
    res = {}
    for arm in ("random", "learned"):
        cfg = api.TreeConfig(crit=api.ENTROPY, K=K, P=P, T=T_max, bins=256, seed=seed, tree=tree,
                             proposal=1 if arm == "learned" else 0, n_seeds=net.n_seeds,
                             mlp_hidden=net.hidden, mlp=net.params if arm == "learned" else None)
        ms, evals, met, nodes = 0.0, 0, 0, 0
        for nodes_d in depths:
            idx = np.concatenate([r for _, r in nodes_d])
            sizes = [len(r) for _, r in nodes_d]
            off = torch.from_numpy(inputs.segment_offsets(sizes)).to(device)
            Xs = Xd.index_select(0, torch.from_numpy(idx).to(device)).contiguous()
            ys = yd.index_select(0, torch.from_numpy(idx).to(device)).contiguous()
            heap = torch.from_numpy(np.array([int(ref["heap"][i]) for i, _ in nodes_d],
                                             np.int32)).to(device)
            lref = np.array([ref["split_loss"][i] for i, _ in nodes_d])
            target = torch.from_numpy((1.0 + tol) * lref).to(device)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = api.search_nodes(Xs, ys, off, heap, cfg, target_loss=target)
            torch.cuda.synchronize()
            ms += 1e3 * (time.perf_counter() - t0)
            ev = out["evals"].cpu().numpy()
            gl = out["gbest_loss"].cpu().numpy()
            evals += int(ev.sum())
            met += int((gl <= (1.0 + tol) * lref).sum())
            nodes += len(nodes_d)
        res[arm] = dict(ms=ms, evals=evals, met=met, nodes=nodes)
        if log:
            log(f"compare[{arm}]: {nodes} nodes, {evals} evaluations, {met} met the target, "
                f"{ms:.1f} ms")
    return res
