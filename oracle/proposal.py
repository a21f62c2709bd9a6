"""Oracle: learned proposal of initial swarm positions (TEST INFRASTRUCTURE).

The paper initialises every particle at random (Sec. III-A) and leaves the
swarm to find the direction.  The learned proposal replaces that random start
by directions predicted from the node's statistics; the swarm, its loss and
its acceptance rule are unchanged, so plain PSO remains the judge of every
direction and the fallback when no network is given.  Nothing here is in the
paper; this module fixes the definitions the GPU path is checked against, in
FP64 NumPy.

Node statistics (classification, K classes, D features), one node:
  mu_d, sigma_d   mean and population standard deviation of feature d;
  pi_k = n_k / n  class proportions; m_k the mean of class k's rows;
  classes are ordered by count, largest first (ties: lower class id first);
  for the c-th class in that order, block c = pi_k (m_k - mu) / sigma;
  the last block v_d = sum_k pi_k Var_k(x_d) / sigma_d^2 (within-class share
  of the variance, in [0, 1]);
  a feature with sigma_d = 0 gets 0 in every block.
The input vector is [block_0 .. block_{K-1}, v] of length K D + D.

Network: h1 = GELU(W1 s + b1), h2 = GELU(W2 h1 + b2), o = W3 h2 + b3 with
GELU(x) = x Phi(x) (Phi the standard normal CDF).  o holds M raw seeds of D
values in the standardised feature space (row-major [M, D]).

Seeds to positions: seed u (standardised space) maps to the raw direction
a_d = u_d / sigma_d (0 where sigma_d = 0), scaled to unit norm, since
u . ((x - mu) / sigma) = sum_d (u_d / sigma_d) x_d - const.  A raw direction
g maps back to the standardised target t_d = g_d sigma_d, unit norm.

Training loss (one sample): with q_i = (u_i . t)^2 for the unit seeds u_i and
b = argmax_i q_i (lowest i on ties), L = sum_i w_i (1 - q_i) with w_b = 1 - eps
and w_i = eps / (M - 1) otherwise (winner-take-all, relaxed so that every
seed keeps a gradient; the sign of a direction does not change its split).

Adam (Kingma and Ba, 2015): m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

SQRT1_2 = 1.0 / math.sqrt(2.0)


# ------------------------------------------------------------------ node statistics
def class_order(counts):
    """Class ids ordered by count, largest first, ties to the lower id."""
    counts = np.asarray(counts)
    return np.lexsort((np.arange(counts.size), -counts))


def node_stats(X, y, K):
    """(s [K D + D], sigma [D]) of one node's rows X [n, D] with labels y."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.int64)
    n, D = X.shape
    s = np.zeros(K * D + D)
    sigma = np.zeros(D)
    if n == 0:
        return s, sigma
    mu = X.mean(axis=0)
    var = ((X - mu) ** 2).mean(axis=0)
    sigma = np.sqrt(var)
    ok = sigma > 0
    counts = np.bincount(y, minlength=K)[:K]
    within = np.zeros(D)
    for c, k in enumerate(class_order(counts)):
        if counts[k] == 0:
            continue
        Xk = X[y == k]
        pk = counts[k] / n
        mk = Xk.mean(axis=0)
        blk = np.zeros(D)
        blk[ok] = pk * (mk[ok] - mu[ok]) / sigma[ok]
        s[c * D:(c + 1) * D] = blk
        within += pk * ((Xk - mk) ** 2).mean(axis=0)
    v = np.zeros(D)
    v[ok] = within[ok] / var[ok]
    s[K * D:] = v
    return s, sigma


# ------------------------------------------------------------------ network
def normal_cdf(x):
    """Phi(x) = erfc(-x / sqrt 2) / 2 (no cancellation in the lower tail)."""
    return 0.5 * erfc(-np.asarray(x, dtype=np.float64) * SQRT1_2)


def gelu(x):
    return x * normal_cdf(x)


def gelu_grad(x):
    """d GELU / dx = Phi(x) + x phi(x)."""
    return normal_cdf(x) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def param_shapes(n_in, hidden, n_out):
    """Shapes of (W1, b1, W2, b2, W3, b3) in their packed order."""
    return [(hidden, n_in), (hidden,), (hidden, hidden), (hidden,), (n_out, hidden), (n_out,)]


def unpack(theta, n_in, hidden, n_out):
    out, o = [], 0
    for shp in param_shapes(n_in, hidden, n_out):
        size = int(np.prod(shp))
        out.append(np.asarray(theta[o:o + size], dtype=np.float64).reshape(shp))
        o += size
    return out


def n_params(n_in, hidden, n_out):
    return sum(int(np.prod(s)) for s in param_shapes(n_in, hidden, n_out))


def forward(theta, S, n_in, hidden, n_out):
    """o [B, n_out] and the cache (z1, h1, z2, h2) for a batch S [B, n_in]."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, hidden, n_out)
    S = np.asarray(S, dtype=np.float64)
    z1 = S @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    o = h2 @ W3.T + b3
    return o, (z1, h1, z2, h2)


def backward(theta, S, cache, d_o, n_in, hidden, n_out):
    """Gradient of sum(d_o * o) with respect to the packed parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, hidden, n_out)
    S = np.asarray(S, dtype=np.float64)
    z1, h1, z2, h2 = cache
    gW3 = d_o.T @ h2
    gb3 = d_o.sum(0)
    d_h2 = d_o @ W3
    d_z2 = d_h2 * gelu_grad(z2)
    gW2 = d_z2.T @ h1
    gb2 = d_z2.sum(0)
    d_h1 = d_z2 @ W2
    d_z1 = d_h1 * gelu_grad(z1)
    gW1 = d_z1.T @ S
    gb1 = d_z1.sum(0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


# ------------------------------------------------------------------ loss
def wta_loss(o, t, M, eps):
    """Per-sample relaxed winner-take-all loss and its gradient d o.

    o [B, M D] raw seeds (standardised space), t [B, D] unit targets."""
    o = np.asarray(o, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B, D = t.shape
    A = o.reshape(B, M, D)
    r = np.sqrt((A * A).sum(-1))
    safe = np.where(r > 0, r, 1.0)
    U = A / safe[..., None]
    c = (U * t[:, None, :]).sum(-1)
    c = np.where(r > 0, c, 0.0)
    q = c * c
    best = np.argmax(q, axis=1)                      # first maximum
    w = np.full((B, M), eps / (M - 1) if M > 1 else 0.0)
    w[np.arange(B), best] = 1.0 - eps if M > 1 else 1.0
    L = (w * (1.0 - q)).sum(1)
    # d(1 - c^2)/dA = -2 c (t - c u) / r
    g = -2.0 * (w * c)[..., None] * (t[:, None, :] - c[..., None] * U) / safe[..., None]
    g = np.where((r > 0)[..., None], g, 0.0)
    return L, g.reshape(B, M * D)


# ------------------------------------------------------------------ seeds and targets
def seeds_to_directions(o_row, sigma, M):
    """Raw unit directions [M, D] from one node's network output [M D]."""
    sigma = np.asarray(sigma, dtype=np.float64)
    D = sigma.size
    U = np.asarray(o_row, dtype=np.float64).reshape(M, D)
    A = np.zeros_like(U)
    ok = sigma > 0
    A[:, ok] = U[:, ok] / sigma[ok]
    nrm = np.sqrt((A * A).sum(1))
    good = nrm > 0
    A[good] /= nrm[good, None]
    return A


def standardized_target(g, sigma):
    """Unit target in the standardised space for a raw direction g."""
    t = np.asarray(g, dtype=np.float64) * np.asarray(sigma, dtype=np.float64)
    n = np.sqrt((t * t).sum())
    return t / n if n > 0 else t


# ------------------------------------------------------------------ optimiser
def adam_step(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
