"""Pins of the learned-proposal oracle (CPU only): node statistics against the
law of total variance and their invariances, GELU against the normal CDF of
scipy, the network and loss gradients against central finite differences,
Adam against its closed form for a constant gradient, and the seed/target
maps against each other and the projection identity they are built on."""
import numpy as np
import pytest
from scipy.stats import norm

from oracle import proposal as PR
from paper_2208_07023_amd import inputs


# ------------------------------------------------------------------ node statistics
def _node(n=900, D=7, K=4, seed=0):
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((K, D)) * 1.5
    y = rng.integers(0, K, n)
    X = means[y] + rng.standard_normal((n, D)) * rng.uniform(0.5, 2.0, D)
    return X, y


def test_stats_law_of_total_variance():
    """sum_c block_c^2 / pi_c + v = 1 per feature (between + within = total)."""
    X, y = _node()
    K, D = 4, X.shape[1]
    s, sigma = PR.node_stats(X, y, K)
    counts = np.bincount(y, minlength=K)
    pis = counts[PR.class_order(counts)] / len(y)
    blocks = s[:K * D].reshape(K, D)
    between = (blocks ** 2 / pis[:, None]).sum(0)
    assert np.allclose(between + s[K * D:], 1.0, rtol=0, atol=1e-12)
    assert np.allclose(blocks.sum(0), 0.0, atol=1e-12)        # sum_k pi_k (m_k - mu) = 0
    assert np.all((s[K * D:] >= 0) & (s[K * D:] <= 1))
    assert np.allclose(sigma, X.std(axis=0), rtol=1e-12)


def test_stats_invariances():
    X, y = _node(seed=1)
    K = 4
    s, sig = PR.node_stats(X, y, K)
    perm = np.random.default_rng(2).permutation(len(y))
    s2, _ = PR.node_stats(X[perm], y[perm], K)
    assert np.allclose(s, s2, atol=1e-12)
    a = np.random.default_rng(3).uniform(0.1, 10, X.shape[1])
    b = np.random.default_rng(4).standard_normal(X.shape[1]) * 100
    s3, sig3 = PR.node_stats(X * a + b, y, K)
    assert np.allclose(s, s3, atol=1e-9)
    assert np.allclose(sig3, sig * a, rtol=1e-9)


def test_stats_class_order_and_degenerate_features():
    rng = np.random.default_rng(5)
    n, D, K = 600, 4, 3
    y = np.array([2] * 300 + [0] * 200 + [1] * 100)
    X = rng.standard_normal((n, D))
    X[:, 1] = 3.0                                    # constant feature
    X[y == 2, 2] += 5.0                              # class 2 separated on feature 2
    s, sigma = PR.node_stats(X, y, K)
    assert sigma[1] == 0 and np.all(s[1::D] == 0)
    # block 0 is class 2 (largest), whose mean on feature 2 sits above mu
    assert s[0 * D + 2] > 0.3 and s[2 * D + 2] < 0
    # equal class means: within share 1 (feature 0 is pure noise up to sampling)
    Xm = np.concatenate([X, 2 * X.mean(0) - X])
    ym = np.concatenate([y, y])
    sm, _ = PR.node_stats(Xm, ym, K)
    assert np.allclose(sm[K * D + 0], 1.0, atol=1e-12)
    # one class only: no between-class part
    s1, _ = PR.node_stats(X, np.zeros(n, dtype=int), K)
    assert np.allclose(s1[K * D:][sigma > 0], 1.0) and np.allclose(s1[D:K * D], 0)


def test_stats_empty_node():
    s, sigma = PR.node_stats(np.zeros((0, 3)), np.zeros(0, dtype=int), 2)
    assert np.all(s == 0) and np.all(sigma == 0)


# ------------------------------------------------------------------ GELU
def test_gelu_against_normal_cdf():
    x = np.linspace(-8, 8, 2001)
    assert np.allclose(PR.gelu(x), x * norm.cdf(x), rtol=5e-14, atol=1e-300)
    assert PR.gelu(0.0) == 0.0
    assert PR.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert PR.gelu(-1.0) == pytest.approx(-0.15865525393145707, rel=1e-14)


def test_gelu_grad_by_central_differences():
    x = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (PR.gelu(x + h) - PR.gelu(x - h)) / (2 * h)
    assert np.allclose(PR.gelu_grad(x), fd, atol=1e-9)


# ------------------------------------------------------------------ network gradient
def test_backward_matches_central_differences():
    n_in, hidden, n_out, B = 5, 4, 6, 3
    rng = np.random.default_rng(7)
    theta = rng.standard_normal(PR.n_params(n_in, hidden, n_out)) * 0.7
    S = rng.standard_normal((B, n_in))
    d_o = rng.standard_normal((B, n_out))
    _, cache = PR.forward(theta, S, n_in, hidden, n_out)
    g = PR.backward(theta, S, cache, d_o, n_in, hidden, n_out)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fp = (PR.forward(theta + e, S, n_in, hidden, n_out)[0] * d_o).sum()
        fm = (PR.forward(theta - e, S, n_in, hidden, n_out)[0] * d_o).sum()
        fd[i] = (fp - fm) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_forward_special_case_linear_region():
    """Zero first two layers: o = W3 GELU(b2) + b3 with h1 = GELU(b1)."""
    n_in, hidden, n_out = 3, 2, 4
    theta = np.zeros(PR.n_params(n_in, hidden, n_out))
    W1, b1, W2, b2, W3, b3 = (np.zeros(s) for s in PR.param_shapes(n_in, hidden, n_out))
    b2[:] = [1.0, -1.0]
    W3[:] = np.arange(8).reshape(4, 2)
    b3[:] = [0.5, 0, 0, -0.5]
    theta = np.concatenate([a.ravel() for a in (W1, b1, W2, b2, W3, b3)])
    o, _ = PR.forward(theta, np.ones((2, n_in)), n_in, hidden, n_out)
    h2 = np.array([norm.cdf(1.0), -norm.cdf(-1.0)])
    assert np.allclose(o, (W3 @ h2 + b3)[None, :].repeat(2, 0), rtol=1e-14)


# ------------------------------------------------------------------ loss
def test_wta_loss_special_cases():
    D, M, eps = 5, 4, 0.1
    t = np.zeros((1, D))
    t[0, 2] = 1.0
    o = np.random.default_rng(1).standard_normal((1, M * D))
    o[0, 1 * D:2 * D] = -3.0 * t[0]                   # seed 1 is -t: q = 1
    L, g = PR.wta_loss(o, t, M, eps)
    A = o.reshape(M, D)
    q = (A @ t[0] / np.linalg.norm(A, axis=1)) ** 2
    want = (eps / (M - 1)) * (1 - q).sum()            # the winner contributes 0
    assert L[0] == pytest.approx(want, rel=1e-13)
    assert np.allclose(g.reshape(M, D)[1], 0.0, atol=1e-15)
    L0, _ = PR.wta_loss(np.tile(t, (1, M)), t, M, eps)
    assert L0[0] == pytest.approx(0.0, abs=1e-15)


def test_wta_gradient_by_central_differences():
    D, M, B, eps = 6, 5, 4, 0.05
    rng = np.random.default_rng(3)
    t = rng.standard_normal((B, D))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    o = rng.standard_normal((B, M * D))
    L, g = PR.wta_loss(o, t, M, eps)
    h = 1e-6
    for b in range(B):
        for i in range(M * D):
            e = np.zeros_like(o)
            e[b, i] = h
            fd = (PR.wta_loss(o + e, t, M, eps)[0][b] - PR.wta_loss(o - e, t, M, eps)[0][b]) / (2 * h)
            assert g[b, i] == pytest.approx(fd, rel=1e-5, abs=1e-8)


# ------------------------------------------------------------------ seeds and targets
def test_seed_and_target_maps_are_inverse_and_preserve_the_split():
    rng = np.random.default_rng(9)
    D = 8
    sigma = rng.uniform(0.2, 5.0, D)
    mu = rng.standard_normal(D)
    g = inputs.random_unit_rows(1, D, seed=10)[0]
    t = PR.standardized_target(g, sigma)
    a = PR.seeds_to_directions(t, sigma, 1)[0]
    assert np.allclose(a, g, atol=1e-14)
    # the standardised projection orders samples like the raw one
    X = rng.standard_normal((50, D)) * sigma + mu
    zs = ((X - mu) / sigma) @ t
    zr = X @ g
    assert np.all(np.argsort(zs) == np.argsort(zr))
    assert np.allclose(np.linalg.norm(PR.seeds_to_directions(rng.standard_normal(3 * D), sigma, 3),
                                      axis=1), 1.0)


# ------------------------------------------------------------------ Adam
def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are g and g^2 at
    every step, so each update is lr g / (|g| + eps)."""
    rng = np.random.default_rng(11)
    g = rng.standard_normal(10)
    theta = rng.standard_normal(10)
    m = np.zeros(10)
    v = np.zeros(10)
    lr, eps = 1e-3, 1e-8
    for step in range(1, 6):
        new, m, v = PR.adam_step(theta, g, m, v, step, lr=lr, eps=eps)
        assert np.allclose(theta - new, lr * g / (np.abs(g) + eps), rtol=1e-9, atol=0)
        theta = new


def test_adam_two_steps_by_hand():
    theta, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    theta, m, v = PR.adam_step(theta, np.array([2.0]), m, v, 1, lr=0.1, b1=0.5, b2=0.75, eps=0.0)
    assert theta[0] == pytest.approx(0.9)                # m^ = 2, v^ = 4
    theta, m, v = PR.adam_step(theta, np.array([-1.0]), m, v, 2, lr=0.1, b1=0.5, b2=0.75, eps=0.0)
    # m = 0.5*1 + 0.5*(-1) = 0 -> no move
    assert m[0] == 0.0 and theta[0] == pytest.approx(0.9)
    assert v[0] == pytest.approx(0.75 * 1.0 + 0.25 * 1.0)
