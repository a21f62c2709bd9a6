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
def _ancestors(tree: dict, leaves, device):
    """For every row's leaf, the node it passed at each depth: [depth, rows]
    (-1 below the row's leaf).  Index bookkeeping on the tree's child lists;
    the routing itself (slm_predict) ran on the device."""
    n = int(tree["n_nodes"])
    parent = np.full(n, -1, np.int64)
    for i in range(n):
        for c in (tree["left"][i], tree["right"][i]):
            if c >= 0:
                parent[c] = i
    depth = tree["depth"][:n].astype(np.int64)
    max_d = int(depth.max()) if n else 0
    par = torch.from_numpy(parent).to(device)
    dep = torch.from_numpy(depth).to(device)
    cur = leaves.to(torch.int64)
    out = torch.full((max_d + 1, cur.numel()), -1, dtype=torch.int64, device=device)
    for d in range(max_d, -1, -1):
        # every row's node is at depth <= d + 1 here: one step up suffices
        cur = torch.where(dep[cur] > d, par[cur], cur)
        out[d] = torch.where(dep[cur] == d, cur, out[d])
    return out


def _node_sets(trees, row_sets, X, device):
    """Rows of every searched node, by depth, over several trees: a list of
    (row indices into X grouped by node, node sizes, (tree, node) pairs).
    Rows are routed through each tree by slm_predict on the device."""
    by_depth = {}
    for b, (tr, rows) in enumerate(zip(trees, row_sets)):
        leaves = api.predict_leaves(tr, X.index_select(0, rows).contiguous())
        anc = _ancestors(tr, leaves, device)
        searched = np.isfinite(tr["split_loss"][:tr["n_nodes"]])
        for d in range(anc.shape[0]):
            ids = anc[d]
            keep = ids >= 0
            if not bool(keep.any()):
                continue
            ids_k = ids[keep]
            rows_k = rows[keep.nonzero().squeeze(1)]
            order = torch.argsort(ids_k, stable=True)
            ids_s, rows_s = ids_k[order], rows_k[order]
            uniq, counts = torch.unique_consecutive(ids_s, return_counts=True)
            uq, ct = uniq.cpu().numpy(), counts.cpu().numpy()
            starts = np.concatenate([[0], np.cumsum(ct)])
            for j, node in enumerate(uq):
                if not searched[node]:
                    continue
                by_depth.setdefault(d, []).append((b, int(node), rows_s[starts[j]:starts[j + 1]]))
    return [by_depth[d] for d in sorted(by_depth)]


def compare_forest(nets: dict, N: int, D: int, K: int, n_trees: int, ref_P: int = 256,
                   ref_T: int = 200, P: int = 64, T_max: int = 50, tol: float = 0.01,
                   max_depth: int = 8, seed: int = 0, mean_std: float = 0.8, clusters: int = 4,
                   device="cuda", log=None):
    """Paired comparison of random and learned (hybrid) swarm starts on the
    nodes of a bootstrap forest.

    A plain forest (n_trees bootstrap trees, P particles, T_max moves) fixes
    the node row sets; a reference search of every node (ref_P particles,
    ref_T moves) fixes each node's reference loss L_ref.  Then, on exactly
    those nodes, batched per depth over all trees, each arm searches with P
    particles until its global-best loss is <= (1 + tol) L_ref or after T_max
    moves: "random" starts all P particles at random (Sec. III-A); "learned_M"
    places the network's M seeds on the first M particles and keeps P - M
    random ones.  Returns per arm: wall ms (including the learned arms'
    statistics and inference), evaluations, nodes that met the target."""
    X, y = cluster_mixture_gpu(N, D, K, clusters, mean_std, seed, device)
    cfg = api.TreeConfig(crit=api.ENTROPY, K=K, max_depth=max_depth, min_node=32, P=P, T=T_max,
                         bins=256, seed=seed, tree=0, use_graph=True)
    forest = api.grow_forest(X, y, cfg, n_trees, return_samples=True)
    trees = [api.forest_tree(forest, b) for b in range(n_trees)]
    samples = forest["samples"].to(torch.int64)
    depths = _node_sets(trees, [samples[b] for b in range(n_trees)], X, device)
    api._forest_ws.clear()
    n_nodes = sum(len(d) for d in depths)
    if log:
        log(f"compare: {n_trees} trees, {n_nodes} searched nodes over {len(depths)} depths")
    batches = []
    for nodes_d in depths:
        idx = torch.cat([r for _, _, r in nodes_d])
        sizes = [int(r.numel()) for _, _, r in nodes_d]
        off = torch.from_numpy(inputs.segment_offsets(sizes)).to(device)
        heap = torch.from_numpy(np.array([b * 4096 + int(trees[b]["heap"][i]) for b, i, _ in nodes_d],
                                         np.int32)).to(device)
        batches.append((idx, off, heap))

    def gathered(idx):
        return X.index_select(0, idx).contiguous(), y.index_select(0, idx).contiguous()

    # reference losses
    ref_cfg = api.TreeConfig(crit=api.ENTROPY, K=K, P=ref_P, T=ref_T, bins=256, seed=seed + 1,
                             tree=0)
    lrefs = []
    t0 = time.perf_counter()
    for idx, off, heap in batches:
        Xs, ys = gathered(idx)
        out = api.search_nodes(Xs, ys, off, heap, ref_cfg)
        lrefs.append(out["gbest_loss"].cpu().numpy())
        del Xs, ys, out
        torch.cuda.empty_cache()
    t_ref = time.perf_counter() - t0
    arms = [("random", None)] + [(f"learned_{m}", nets[m]) for m in sorted(nets)]
    res = {"nodes": n_nodes, "reference_s": t_ref}
    for name, net in arms:
        acfg = api.TreeConfig(crit=api.ENTROPY, K=K, P=P, T=T_max, bins=256, seed=seed, tree=0,
                              proposal=0 if net is None else 1,
                              n_seeds=net.n_seeds if net else 64,
                              mlp_hidden=net.hidden if net else 256,
                              mlp=net.params if net else None)
        ms, evals, met, at_max = 0.0, 0, 0, 0
        for (idx, off, heap), lref in zip(batches, lrefs):
            Xs, ys = gathered(idx)
            target = torch.from_numpy((1.0 + tol) * lref).to(device)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = api.search_nodes(Xs, ys, off, heap, acfg, target_loss=target)
            torch.cuda.synchronize()
            ms += 1e3 * (time.perf_counter() - t0)
            ev = out["evals"].cpu().numpy()
            gl = out["gbest_loss"].cpu().numpy()
            evals += int(ev.sum())
            met += int((gl <= (1.0 + tol) * lref).sum())
            at_max += int((ev >= T_max + 1).sum())
            del Xs, ys, out
        res[name] = dict(ms=ms, evals=evals, met=met, hit_T_max=at_max)
        if log:
            log(f"compare[{name}]: {evals} evaluations, {met}/{n_nodes} met the target, "
                f"{at_max} ran to T_max, {ms:.1f} ms")
    r = res["random"]
    for name, _ in arms[1:]:
        l = res[name]
        l["speedup_wall"] = r["ms"] / max(1e-9, l["ms"])
        l["speedup_evals"] = r["evals"] / max(1, l["evals"])
    return res
