"""GPU parity of the learned-proposal kernels and of the node-batch search,
through the C ABI, against the FP64 oracle.

Bars (the kernels compute in FP32 where the oracle uses FP64, except the
statistics' sums and the seed map, which are FP64):
* node statistics: |GPU - oracle| <= 2e-6 (FP32 outputs of FP64 sums);
* network forward: |o - o_64| <= 1e-4 RMS(o_64) (FP32), <= 4e-2 RMS with
  BF16 inference (both operands of every product rounded to 8 bits);
* backward: every parameter block's gradient within 1e-4 of the oracle's,
  relative to the block's norm;
* loss and its gradient within 1e-5; Adam within 1e-6 relative;
* seeds to directions within 1e-12 (FP64 from FP32 inputs);
* the node-batch search: without targets bit-identical to the tree's own
  root search; with targets its stopping evaluation and global best are those
  of the same search cut after that many evaluations.
"""
import numpy as np
import pytest
import torch

from oracle import proposal as PR
from oracle import screen as SC
from paper_2208_07023_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


# ------------------------------------------------------------------ statistics
@pytest.mark.parametrize("K,D,bf16,sizes", [(3, 7, False, [500, 0, 3000, 1]),
                                            (5, 128, False, [5000, 2049]),
                                            (5, 64, True, [100, 4100]),
                                            (16, 16, False, [7000])])
def test_node_stats_match_oracle(gpu_lib, K, D, bf16, sizes):
    api = gpu_lib
    off = inputs.segment_offsets(sizes)
    N = int(off[-1])
    rng = np.random.default_rng(K * D)
    means = rng.standard_normal((K, D)) * 2
    y = rng.integers(0, K, N).astype(np.int32)
    y[: N // 3] = 0                          # uneven classes
    X = (means[y] + rng.standard_normal((N, D)) * rng.uniform(0.5, 2, D) + 3).astype(np.float32)
    X[:, 0] = 1.5                            # a constant feature
    if bf16:
        X = SC.bf16_round(X)
    Xd = _t(X).to(torch.bfloat16) if bf16 else _t(X)
    stats, sigma = api.node_stats(Xd, _t(y), K, _t(off))
    stats, sigma = stats.cpu().numpy(), sigma.cpu().numpy()
    for j in range(len(sizes)):
        r0, r1 = off[j], off[j + 1]
        s_ref, g_ref = PR.node_stats(X[r0:r1], y[r0:r1], K)
        assert np.allclose(stats[j], s_ref, rtol=0, atol=2e-6), j
        assert np.allclose(sigma[j], g_ref, rtol=2e-6, atol=1e-7), j


# ------------------------------------------------------------------ network
def _params(I, H, O, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for shp in PR.param_shapes(I, H, O):
        fan = shp[1] if len(shp) == 2 else 1
        parts.append((rng.standard_normal(shp) * scale / np.sqrt(fan)).ravel())
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("I,H,O,B", [(768, 256, 8192, 70), (19, 8, 12, 5), (130, 64, 200, 129)])
def test_mlp_forward_matches_oracle(gpu_lib, I, H, O, B):
    api = gpu_lib
    th = _params(I, H, O, seed=I + O)
    S = np.random.default_rng(1).standard_normal((B, I)).astype(np.float32)
    assert api.mlp_param_count(I, H, O) == th.size
    o, cache = api.mlp_forward(_t(th), I, H, O, _t(S))
    ob, _ = api.mlp_forward(_t(th), I, H, O, _t(S), bf16=True)
    ref, rc = PR.forward(th.astype(np.float64), S, I, H, O)
    rms = np.sqrt(np.mean(ref ** 2))
    assert np.max(np.abs(o.cpu().numpy() - ref)) <= 1e-4 * rms
    assert np.max(np.abs(ob.cpu().numpy() - ref)) <= 4e-2 * rms
    c = cache.cpu().numpy()                            # z1, h1, z2, h2 blocks
    for i in range(4):
        assert np.allclose(c[i], rc[i], atol=1e-4 * np.sqrt(np.mean(rc[i] ** 2)) + 1e-6), i


@pytest.mark.parametrize("I,H,O,B", [(768, 256, 8192, 64), (19, 8, 12, 5), (130, 64, 200, 129)])
def test_mlp_backward_matches_oracle(gpu_lib, I, H, O, B):
    api = gpu_lib
    th = _params(I, H, O, seed=I + 7)
    rng = np.random.default_rng(2)
    S = rng.standard_normal((B, I)).astype(np.float32)
    d_o = rng.standard_normal((B, O)).astype(np.float32)
    o, cache = api.mlp_forward(_t(th), I, H, O, _t(S))
    g = api.mlp_backward(_t(th), I, H, O, _t(S), cache, _t(d_o)).cpu().numpy()
    _, rc = PR.forward(th.astype(np.float64), S, I, H, O)
    ref = PR.backward(th.astype(np.float64), S, rc, d_o.astype(np.float64), I, H, O)
    o0 = 0
    for shp in PR.param_shapes(I, H, O):
        n = int(np.prod(shp))
        a, b = g[o0:o0 + n], ref[o0:o0 + n]
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-6, shp
        o0 += n


def test_wta_loss_matches_oracle(gpu_lib):
    api = gpu_lib
    B, M, D, eps = 37, 64, 128, 0.05
    rng = np.random.default_rng(3)
    o = rng.standard_normal((B, M * D)).astype(np.float32)
    o[0, :D] = 0.0                            # a zero seed
    t = rng.standard_normal((B, D))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    t = t.astype(np.float32)
    o[1, 2 * D:3 * D] = -2.5 * t[1]           # a seed on the target's line
    L, g = api.wta_loss(_t(o), _t(t), M, eps)
    Lr, gr = PR.wta_loss(o, t, M, eps)
    assert np.allclose(L.cpu().numpy(), Lr, atol=1e-5)
    assert np.allclose(g.cpu().numpy(), gr, atol=1e-5)
    _, g2 = api.wta_loss(_t(o), _t(t), M, eps, scale=1.0 / B)
    assert np.allclose(g2.cpu().numpy(), gr / B, atol=1e-5 / B)


def test_proposal_targets_match_oracle(gpu_lib):
    api = gpu_lib
    rng = np.random.default_rng(8)
    n, D = 33, 128
    g = inputs.random_unit_rows(n, D, seed=9).astype(np.float32)
    sigma = rng.uniform(0.05, 4, (n, D)).astype(np.float32)
    sigma[0, :5] = 0
    t = api.proposal_targets(_t(g), _t(sigma)).cpu().numpy()
    for i in range(n):
        assert np.allclose(t[i], PR.standardized_target(g[i], sigma[i]), rtol=0, atol=2e-7)


def test_adam_matches_oracle(gpu_lib):
    api = gpu_lib
    n = 10007
    rng = np.random.default_rng(4)
    p = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    P_, M_, V_ = _t(p), _t(m), _t(v)
    pr, mr, vr = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for step in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32)
        api.adam_step(P_, _t(g), M_, V_, lr=1e-3, step=step)
        pr, mr, vr = PR.adam_step(pr, g.astype(np.float64), mr, vr, step)
    assert np.allclose(P_.cpu().numpy(), pr, rtol=1e-6, atol=1e-7)


def test_seeds_match_oracle(gpu_lib):
    api = gpu_lib
    nn, M, D, P = 3, 5, 9, 7
    rng = np.random.default_rng(5)
    o = rng.standard_normal((nn, M * D)).astype(np.float32)
    o[1, :D] = 0.0                            # zero seed: particle keeps its start
    sigma = rng.uniform(0.1, 3, (nn, D)).astype(np.float32)
    sigma[2, 3] = 0.0
    sw = api.pso_alloc(nn, P, D, node_id=np.arange(nn))
    api.pso_init(sw, seed=1, tree=0)
    x0 = sw.x.cpu().numpy().copy()
    api.proposal_seeds(_t(o), _t(sigma), M, sw)
    x = sw.x.cpu().numpy().reshape(nn, P, D)
    for j in range(nn):
        A = PR.seeds_to_directions(o[j], sigma[j], M)
        for i in range(M):
            if j == 1 and i == 0:
                assert np.array_equal(x[j, i], x0.reshape(nn, P, D)[j, i])
            else:
                assert np.allclose(x[j, i], A[i], rtol=0, atol=1e-12)
        assert np.array_equal(x[j, M:], x0.reshape(nn, P, D)[j, M:])
    assert np.array_equal(sw.pbest.cpu().numpy(), sw.x.cpu().numpy())
    assert np.array_equal(sw.W.cpu().numpy(), sw.x.cpu().numpy().astype(np.float32))


# ------------------------------------------------------------------ node-batch search
def test_search_nodes_equals_tree_root_search(gpu_lib):
    """One node searched alone reproduces the tree's root search bit for bit
    (same random stream, same kernels)."""
    api = gpu_lib
    X, y = inputs.cluster_mixture(6000, 16, 3, seed=21)
    cfg = api.TreeConfig(crit=api.GINI, K=3, max_depth=1, min_node=2, P=48, T=7, bins=64, seed=4)
    tr = api.grow_tree(_t(X), _t(y), cfg)
    out = api.search_nodes(_t(X), _t(y), _t(np.array([0, 6000], np.int64)),
                           _t(np.array([0], np.int32)), cfg)
    assert out["gbest_loss"].cpu().numpy()[0] == tr["split_loss"][0]
    assert np.array_equal(out["gbest"].cpu().numpy()[0].astype(np.float32), tr["w"][0])
    assert out["gbest_thr"].cpu().numpy()[0] == tr["thr"][0]
    assert out["evals"].cpu().numpy()[0] == cfg.T + 1


def test_search_nodes_stops_at_the_target(gpu_lib):
    api = gpu_lib
    X, y = inputs.cluster_mixture(8000, 12, 3, seed=22)
    off = np.array([0, 4000, 6500, 8000], np.int64)
    nid = np.array([0, 1, 2], np.int32)
    cfg = api.TreeConfig(crit=api.ENTROPY, K=3, P=32, T=12, bins=64, seed=6)
    full = [api.search_nodes(_t(X), _t(y), _t(off), _t(nid),
                             api.TreeConfig(**{**cfg.__dict__, "T": t}))["gbest_loss"].cpu().numpy()
            for t in range(cfg.T + 1)]
    hist = np.stack(full)                     # [T+1 evaluations, nodes]
    # targets: reached after 1, after 5 evaluations, and never
    target = np.array([hist[0, 0], hist[4, 1], -1.0])
    out = api.search_nodes(_t(X), _t(y), _t(off), _t(nid), cfg, target_loss=_t(target))
    ev = out["evals"].cpu().numpy()
    want = [int(np.argmax(hist[:, j] <= target[j])) + 1 if np.any(hist[:, j] <= target[j])
            else cfg.T + 1 for j in range(3)]
    assert ev.tolist() == want
    gl = out["gbest_loss"].cpu().numpy()
    for j in range(3):
        assert gl[j] == hist[want[j] - 1, j]


def _balanced_signs(n, D, rng):
    """[n, D] of +-1 with exactly n/2 of each sign per column: every column has
    mean 0 and variance 1 exactly, so sigma = 1 on both sides."""
    X = np.empty((n, D), np.float32)
    for d in range(D):
        X[:, d] = rng.permutation(np.repeat(np.array([1.0, -1.0], np.float32), n // 2))
    return X


def test_learned_start_search_matches_oracle(gpu_lib):
    """slm_search_nodes with the learned start (proposal 1: node statistics,
    BF16 network inference, seeds, then the swarm) against the oracle's steps
    in the same order (oracle.proposal.node_stats -> forward ->
    seeds_to_directions -> oracle.pso.run_pso with those seeds, T = 0).

    The network's weights are zero and its output biases are +-1 on four
    coordinates per seed (bfloat16 values), and every data column is a
    balanced +-1 column (sigma = 1 exactly): the seeds are then +-1/2 on four
    coordinates on both sides, every projection is exact in FP32, and the
    first evaluation's global best -- direction, loss, split and threshold --
    must agree bit for bit.  The seeds themselves are compared with the
    oracle's to 1e-12 through the separate calls (node statistics, forward,
    seed map) that the search composes."""
    from oracle import pso as OP
    from oracle import split as OS
    from oracle import tree as OT
    api = gpu_lib
    D, K, M, H = 8, 2, 8, 16
    rng = np.random.default_rng(41)
    sizes = [1000, 600]
    Xs, ys = [], []
    for n in sizes:
        X = _balanced_signs(n, D, rng)
        y = ((X[:, 0] + X[:, 1] + X[:, 2] + 0.5 * rng.standard_normal(n)) > 0).astype(np.int32)
        Xs.append(X)
        ys.append(y)
    X, y = np.concatenate(Xs), np.concatenate(ys)
    off = inputs.segment_offsets(sizes)
    n_in, n_out = (K + 1) * D, M * D
    theta = np.zeros(PR.n_params(n_in, H, n_out), np.float32)
    b3 = np.zeros((M, D), np.float32)
    for m in range(M):                 # distinct sign patterns on four coordinates
        cols = rng.choice(D, 4, replace=False)
        b3[m, cols] = rng.choice([-1.0, 1.0], 4)
    theta[-n_out:] = b3.ravel()
    cfg = api.TreeConfig(crit=api.GINI, K=K, P=M, T=0, bins=64, seed=3, proposal=1, n_seeds=M,
                         mlp_hidden=H, mlp=_t(theta))
    node_id = np.array([5, 9], np.int32)
    out = api.search_nodes(_t(X), _t(y), _t(off), _t(node_id), cfg)
    prm = OT.TreeParams(crit=OS.GINI, K=K, P=M, T=0, bins=64, seed=3)
    for j in range(len(sizes)):
        Xn, yn = X[off[j]:off[j + 1]], y[off[j]:off[j + 1]]
        s, sigma = PR.node_stats(Xn, yn, K)
        assert np.array_equal(sigma, np.ones(D))
        o, _ = PR.forward(theta.astype(np.float64), s[None, :], n_in, H, n_out)
        seeds = PR.seeds_to_directions(o[0], sigma, M)
        assert np.all(np.isin(np.abs(seeds), [0.0, 0.5]))
        ref = OP.run_pso(OT.evaluate_node(Xn, yn, prm), M, D, 0, prm.omega, prm.c1, prm.c2,
                         prm.seed, prm.tree, int(node_id[j]), x0=seeds)
        assert out["gbest_loss"].cpu().numpy()[j] == ref["loss"]
        assert np.array_equal(out["gbest"].cpu().numpy()[j], ref["gbest"])
        assert out["gbest_split"].cpu().numpy()[j] == ref["split"]
        assert out["gbest_thr"].cpu().numpy()[j] == ref["thr"]
        assert out["evals"].cpu().numpy()[j] == 1
    # the steps the search composes, called one by one, place the same seeds
    st, sg = api.node_stats(_t(X), _t(y), K, _t(off))
    o_gpu, _ = api.mlp_forward(_t(theta), n_in, H, n_out, st, bf16=True)
    sw = api.pso_alloc(len(sizes), M, D, node_id=node_id)
    api.pso_init(sw, seed=3, tree=0)
    api.proposal_seeds(o_gpu, sg, M, sw)
    x = sw.x.cpu().numpy().reshape(len(sizes), M, D)
    for j in range(len(sizes)):
        Xn, yn = X[off[j]:off[j + 1]], y[off[j]:off[j + 1]]
        s, sigma = PR.node_stats(Xn, yn, K)
        o, _ = PR.forward(theta.astype(np.float64), s[None, :], n_in, H, n_out)
        assert np.allclose(x[j], PR.seeds_to_directions(o[0], sigma, M), rtol=0, atol=1e-12)
