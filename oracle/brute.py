"""Brute-force split losses in exact arithmetic (tiny inputs only).

For every candidate threshold t the two sides {z < t} and {z >= t} are formed
directly (Sec. II-A, Eqs. (3)-(4)) and the weighted child impurity is computed
from its textbook definition:
* Gini: sum over sides of n_c/n * (1 - sum_k (n_ck/n_c)^2), in Fractions;
* squared error: sum over sides of sum_i (y_i - mean_c)^2, divided by n, in
  Fractions built from the exact binary values of y;
* entropy: sum over sides of n_c/n * (-sum_k p_k log2 p_k), in 60-digit Decimal.
No histogram, prefix sum or closed-form rearrangement is used, so these serve
as an independent check of oracle.split.
"""
from __future__ import annotations

from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

GINI, ENTROPY, MSE = 0, 1, 2


def _gini_side(labels, K):
    n = len(labels)
    if n == 0:
        return Fraction(0)
    cnt = [0] * K
    for k in labels:
        cnt[int(k)] += 1
    return Fraction(n) * (1 - sum(Fraction(c, n) ** 2 for c in cnt))


def _sse_side(ys):
    if len(ys) == 0:
        return Fraction(0)
    fr = [Fraction(float(v)) for v in ys]
    m = sum(fr) / len(fr)
    return sum((v - m) ** 2 for v in fr)


def _entropy_side(labels, K):
    getcontext().prec = 60
    n = len(labels)
    if n == 0:
        return Decimal(0)
    cnt = [0] * K
    for k in labels:
        cnt[int(k)] += 1
    ln2 = Decimal(2).ln()
    h = Decimal(0)
    for c in cnt:
        if c:
            p = Decimal(c) / Decimal(n)
            h -= p * (p.ln() / ln2)
    return Decimal(n) * h


def split_loss(z, target, t, crit, K=0):
    """Exact weighted child impurity of the split at threshold t, or None if a
    side is empty."""
    z = np.asarray(z)
    target = np.asarray(target)
    right = [i for i in range(z.size) if z[i] >= t]
    left = [i for i in range(z.size) if not z[i] >= t]
    if not left or not right:
        return None
    n = z.size
    if crit == GINI:
        return (_gini_side(target[left], K) + _gini_side(target[right], K)) / n
    if crit == MSE:
        return (_sse_side(target[left]) + _sse_side(target[right])) / n
    return (_entropy_side(target[left], K) + _entropy_side(target[right], K)) / Decimal(n)


def best_over(z, target, thresholds, crit, K=0):
    """Exact losses for each candidate threshold (None where invalid), the exact
    minimum, and the indices of all candidates attaining it."""
    losses = [split_loss(z, target, t, crit, K) for t in thresholds]
    valid = [l for l in losses if l is not None]
    if not valid:
        return losses, None, []
    best = min(valid)
    return losses, best, [i for i, l in enumerate(losses) if l is not None and l == best]


def bins_by_counting(z32, edges):
    """bin(z) = number of edges <= z, counted edge by edge."""
    out = np.zeros(len(z32), dtype=np.int64)
    for i, v in enumerate(z32):
        out[i] = sum(1 for e in edges if e <= v)
    return out
