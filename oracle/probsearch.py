"""Oracle: probabilistic search for projection directions (Sec. II-B, the
original SLM's search, Eqs. (5)-(8)), as an alternative proposal over the same
projection and threshold scan (test infrastructure only).

The basis vectors e_d are ranked by their DFT loss (oracle.dft; most
discriminant first).  A candidate direction is a combination of the first R
ranked vectors with integer coefficients: the coefficient of rank d is drawn
with probability P_d, and then uniformly among +-1, ..., +-floor(A_d)
(Eq. (7)); the other coefficients are 0.  Each search iteration draws P
candidates per node, evaluates them and keeps the best seen so far.

Readings (the paper leaves the constants to its reference):
* P_d and floor(A_d) are inputs (tables over the R ranks), so both sides use
  the same values; the library's callers build them as A_d = alpha0
  exp(-alpha (d - 1)), alpha = ln(alpha0) / (R - 1) (A falls from alpha0 at
  rank 1 to 1 at rank R, Eq. (8)), and P_d = A_d / alpha0 (the selection
  probability decays with the same exponential);
* the pruning of highly correlated vectors serves the original SLM, which
  keeps several projections per node; the accelerated binary tree keeps the
  single best, so it is not applied;
* Eq. (7) lists 0 among the values; here the draw with probability P_d
  decides whether a coefficient is used, and a used one is nonzero;
* a candidate whose draws select no coefficient takes +1 on rank 1;
* the candidate is scaled to unit norm (Eq. (2)); its squared norm is an
  integer, so the direction is the exact integer vector divided by the
  correctly rounded square root;
* random numbers: one Philox4x32-10 call per (particle, rank) with counter
  (p * R + d, 0x40000000 + t, node, tree) and the seed as key; word 0 decides
  the selection (u24(w0) < P_d), word 1 the value index
  k = floor(u24(w1) * 2 m), m = floor(A_d): coefficient k + 1 for k < m, else
  -(k - m + 1).
"""
from __future__ import annotations

import math

import numpy as np

from .philox import philox4x32_10, seed_key, u24

STREAM = 0x40000000


def tables(R: int, alpha0: float):
    """(P_d [R] float64, floor(A_d) [R] int32) of the reading above."""
    d = np.arange(R, dtype=np.float64)
    alpha = math.log(alpha0) / (R - 1) if R > 1 else 0.0
    A = alpha0 * np.exp(-alpha * d)
    return A / alpha0, np.maximum(1, np.floor(A + 1e-9)).astype(np.int32)


def coefficients(seed, tree, node, t, P, ranks, pd, amax):
    """Integer coefficients [P, D] of the P candidates of one node at
    iteration t; ranks [>= R]: feature indices from most to least
    discriminant."""
    R = len(pd)
    ranks = np.asarray(ranks, dtype=np.int64)
    D = None
    ctr = np.array([[p * R + d, STREAM + t, node, tree] for p in range(P) for d in range(R)],
                   dtype=np.uint64).reshape(P, R, 4)
    w = philox4x32_10(ctr, seed_key(seed))
    sel = u24(w[..., 0]) < np.asarray(pd)[None, :]
    m = np.asarray(amax, dtype=np.int64)[None, :]
    k = np.floor(u24(w[..., 1]) * (2 * m)).astype(np.int64)
    val = np.where(k < m, k + 1, -(k - m + 1))
    coef = np.where(sel, val, 0)
    none = ~sel.any(axis=1)
    coef[none, 0] = 1
    return coef, ranks[:R]


def candidates(seed, tree, node, t, P, D, ranks, pd, amax):
    """Unit directions [P, D] (float64) of the P candidates."""
    coef, rk = coefficients(seed, tree, node, t, P, ranks, pd, amax)
    x = np.zeros((P, D))
    x[:, rk] = coef
    s = np.zeros(P)
    for j in range(x.shape[1]):          # squared norm in dimension order
        s = s + x[:, j] * x[:, j]
    return x / np.sqrt(s)[:, None]


def run_search(evaluate, P, D, T, seed, tree, node, ranks, pd, amax):
    """T + 1 iterations of P candidates; returns dict(gbest, loss, split, thr,
    p, evals, history) like oracle.pso.run_pso: the best candidate seen (the
    first on ties, in iteration then particle order)."""
    best = dict(gbest=None, loss=np.inf, split=-1, thr=np.float32(np.inf), p=-1)
    history = []
    for t in range(T + 1):
        x = candidates(seed, tree, node, t, P, D, ranks, pd, amax)
        loss, split, thr = evaluate(x.astype(np.float32))[:3]
        p = int(np.argmin(loss))
        if loss[p] < best["loss"]:
            best.update(gbest=x[p].copy(), loss=float(loss[p]), split=int(split[p]),
                        thr=np.float32(thr[p]), p=p)
        history.append(best["loss"])
    best["evals"] = T + 1
    best["history"] = history
    return best
