"""End to end on the GPU: harvest (statistics, global best) pairs from plain-PSO
trees, train the proposal network with the library's kernels, and compare
learned and random swarm starts on held-out nodes at equal loss targets.

What is asserted: the pairs are well formed, training lowers the loss and
fits its training pairs better than the untrained network, the learned start
is bit-reproducible, and the learned search meets the loss target on a share
of nodes comparable to the random one.  How much the learned start saves is
printed (it depends on how much of a node's best direction its class
statistics determine; the comparison is measured, not assumed).
"""
import numpy as np
import pytest
import torch

from paper_2208_07023_amd import inputs
from paper_2208_07023_amd import proposal as PL

pytestmark = pytest.mark.gpu


def test_harvest_train_compare_small(gpu_lib):
    api = gpu_lib
    D, K, M, H = 16, 3, 16, 64
    S, G, T = PL.harvest(24, D, K, 4000, 30000, seed=3, P=32, T=20, max_depth=5, clusters=1)
    n = S.shape[0]
    assert n > 100 and S.shape[1] == (K + 1) * D and T.shape == (n, D)
    tn = T.norm(dim=1).cpu().numpy()
    assert np.allclose(tn[tn > 0], 1.0, atol=1e-5)
    net0 = PL.Net(PL.init_params((K + 1) * D, H, M * D, 0), (K + 1) * D, H, M * D, M, D, K)
    net, hist = PL.train(S, T, D, K, n_seeds=M, hidden=H, epochs=30, batch=128)
    print(f"pairs {n}; loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    assert hist[-1] < 0.8 * hist[0]
    c0, c1 = PL.mean_best_cos2(net0, S, T), PL.mean_best_cos2(net, S, T)
    print(f"mean best cos^2 on the training pairs: untrained {c0:.3f}, trained {c1:.3f}")
    assert c1 > c0

    X, y = inputs.cluster_mixture(30000, D, K, clusters_per_class=1, mean_std=0.6, seed=99)
    res = PL.compare_starts(net, X, y, K, ref_P=128, ref_T=60, P=M, T_max=30, max_depth=5)
    r, l = res["random"], res["learned"]
    print(f"random: {r}\nlearned: {l}\nevaluations random/learned = "
          f"{r['evals'] / max(1, l['evals']):.2f}, wall = {r['ms'] / max(1e-9, l['ms']):.2f}")
    assert r["nodes"] == l["nodes"] > 0
    assert l["met"] >= 0.5 * r["met"]
    # the learned start is deterministic
    res2 = PL.compare_starts(net, X, y, K, ref_P=128, ref_T=60, P=M, T_max=30, max_depth=5)
    assert res2["learned"]["evals"] == l["evals"] and res2["learned"]["met"] == l["met"]
