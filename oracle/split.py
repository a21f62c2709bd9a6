"""Oracle: projection and best-threshold search of a projected 1-D feature.

Paper passages followed:
* Sec. II-A, Eqs. (1)-(2): a projected feature is f(a) = a^T x for a unit
  direction a.
* Sec. II-A, Eqs. (3)-(4): a threshold t_b splits the samples into the set with
  a^T x >= t_b (right) and the set with a^T x < t_b (left).
* Sec. II-A and Sec. III-B: a direction is scored by the loss of its best
  threshold (the "DFT loss"; its reference is not in the paper).  This build
  reads that loss as the sample-weighted impurity of the two children under the
  Gini, entropy (base 2) or squared-error criterion, minimised over candidate
  thresholds.

Two candidate-threshold sets are defined (the paper names neither):
* exact: a boundary between consecutive distinct sorted values; the threshold
  is the smallest value sent right;
* histogram: B-1 float32 edges e_j = zmin + j * ((zmax - zmin) / B), each
  operation rounded to float32, j = 1..B-1; a sample's bin is the number of
  edges <= z, split b sends bins < b left and uses threshold e_b, so that
  "z >= e_b" and "bin >= b" select the same samples.

Ties between candidates go to the smallest split index; a candidate needs at
least one sample on each side.  Everything is FP64 except the float32 edge rule,
which is part of the candidate definition.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

GINI, ENTROPY, MSE = 0, 1, 2


# ---------------------------------------------------------------- projection
def project(X, W):
    """Z[i, p] = sum_d X[i, d] * W[p, d] in FP64 (Eq. (1)).

    X and W are upcast exactly from their stored precision (float32 or the
    bfloat16 values widened to float32)."""
    return np.asarray(X, dtype=np.float64) @ np.asarray(W, dtype=np.float64).T


def project_fsum(X, W):
    """Correctly rounded FP64 projection via math.fsum (tiny inputs only)."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    out = np.empty((X.shape[0], W.shape[0]))
    for i in range(X.shape[0]):
        for p in range(W.shape[0]):
            out[i, p] = math.fsum(X[i] * W[p])
    return out


# ---------------------------------------------------------------- binning
def hist_edges(zmin, zmax, B: int) -> np.ndarray:
    """The B-1 float32 edges e_1..e_{B-1}; every operation rounded to float32."""
    zmin = np.float32(zmin)
    zmax = np.float32(zmax)
    r = np.float32(zmax - zmin)
    delta = np.float32(r / np.float32(B))
    j = np.arange(1, B, dtype=np.float32)
    prod = (j * delta).astype(np.float32)
    return (zmin + prod).astype(np.float32)


def hist_bins(z32, zmin, zmax, B: int) -> np.ndarray:
    """bin(z) = #{ j : e_j <= z } in [0, B-1] (edges are non-decreasing)."""
    e = hist_edges(zmin, zmax, B)
    return np.searchsorted(e, np.asarray(z32, dtype=np.float32), side="right").astype(np.int64)


# ---------------------------------------------------------------- criteria
def _nlog2n(n):
    n = np.asarray(n, dtype=np.float64)
    out = np.zeros_like(n)
    pos = n > 0
    out[pos] = n[pos] * np.log2(n[pos])
    return out


def gini_children(cl, cr):
    """Weighted Gini of the children, n-normalised.

    With A_c = sum_k n_ck^2 (exact integer), s = A_L/n_L + A_R/n_R and
    n = n_L + n_R, the weighted impurity n_L/n (1 - A_L/n_L^2) + n_R/n (1 -
    A_R/n_R^2) equals (n - s)/n.  Evaluated as: two divisions, one add, one
    subtract, one divide, each rounded once in FP64.  Invalid (an empty side)
    gives +inf."""
    cl = np.asarray(cl, dtype=np.int64)
    cr = np.asarray(cr, dtype=np.int64)
    nL = cl.sum(-1)
    nR = cr.sum(-1)
    AL = (cl * cl).sum(-1).astype(np.float64)
    AR = (cr * cr).sum(-1).astype(np.float64)
    n = (nL + nR).astype(np.float64)
    valid = (nL > 0) & (nR > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = AL / nL.astype(np.float64) + AR / nR.astype(np.float64)
        loss = (n - s) / n
    return np.where(valid, loss, np.inf)


def gini_node(c):
    """Gini impurity of one node from its class counts, in the same form."""
    c = np.asarray(c, dtype=np.int64)
    n = float(c.sum())
    if n == 0:
        return 0.0
    A = float((c * c).sum())
    return (n - A / n) / n


def entropy_children(cl, cr):
    """Weighted base-2 entropy of the children.

    T_c = n_c log2 n_c - sum_k n_ck log2 n_ck (0 log 0 = 0) equals n_c times
    the child's entropy; the loss is (T_L + T_R) / n.  Empty side: +inf."""
    cl = np.asarray(cl, dtype=np.int64)
    cr = np.asarray(cr, dtype=np.int64)
    nL = cl.sum(-1)
    nR = cr.sum(-1)
    TL = _nlog2n(nL) - _nlog2n(cl).sum(-1)
    TR = _nlog2n(nR) - _nlog2n(cr).sum(-1)
    n = (nL + nR).astype(np.float64)
    valid = (nL > 0) & (nR > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        loss = (TL + TR) / n
    return np.where(valid, loss, np.inf)


def entropy_node(c):
    c = np.asarray(c, dtype=np.int64)
    n = c.sum()
    if n == 0:
        return 0.0
    return float((_nlog2n(n) - _nlog2n(c).sum()) / n)


def mse_children(nL, s1L, s2L, nR, s1R, s2R):
    """Weighted squared error of the children: (SSE_L + SSE_R) / n with
    SSE_c = S2_c - S1_c^2 / n_c (S1 = sum y, S2 = sum y^2).  Empty side: +inf."""
    nL = np.asarray(nL, dtype=np.float64)
    nR = np.asarray(nR, dtype=np.float64)
    valid = (nL > 0) & (nR > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        sseL = s2L - (s1L * s1L) / nL
        sseR = s2R - (s1R * s1R) / nR
        loss = (sseL + sseR) / (nL + nR)
    return np.where(valid, loss, np.inf)


def mse_node(y):
    y = np.asarray(y, dtype=np.float64)
    if y.size == 0:
        return 0.0
    s1, s2 = exact_sum(y), exact_sum_sq(y)
    return (s2 - s1 * s1 / y.size) / y.size


# ---------------------------------------------------------------- exact sums
def _scaled_ints(vals, square: bool):
    """Exact integer images of vals (or vals^2) on a common power-of-two scale."""
    reps = []
    for v in vals:
        m, e = math.frexp(float(v))
        M = int(math.ldexp(m, 53))
        E = e - 53
        if square:
            M, E = M * M, 2 * E
        reps.append((M, E))
    if not reps:
        return [], 0
    emin = min(E for _, E in reps)
    return [M << (E - emin) for M, E in reps], emin


def _to_float(P: int, emin: int) -> float:
    """Correctly rounded float of P * 2^emin (Python int division rounds once)."""
    if emin >= 0:
        return float(P << emin)
    return P / (1 << (-emin))


def exact_prefix(vals, cuts, square=False):
    """Correctly rounded sums of vals[:c] (or of their squares) for each c in cuts."""
    ints, emin = _scaled_ints(vals, square)
    pref = [0] + list(itertools.accumulate(ints))
    return np.array([_to_float(pref[c], emin) for c in cuts], dtype=np.float64)


def exact_sum(vals):
    return float(exact_prefix(vals, [len(vals)])[0])


def exact_sum_sq(vals):
    return float(exact_prefix(vals, [len(vals)], square=True)[0])


# ---------------------------------------------------------------- scans
NO_SPLIT = -1


def scan_hist(z32, target, B: int, crit: int, K: int = 0):
    """Histogram scan of one projected feature (one node, one particle).

    Returns dict(split, loss, thr, counts, sums): split = b in 1..B-1 or -1;
    thr = e_b (float32) or +inf; counts [B, K] int64 (classification) or [B]
    (regression); sums [B, 2] (sum y, sum y^2; regression only)."""
    z32 = np.asarray(z32, dtype=np.float32)
    n = z32.size
    res = dict(split=NO_SPLIT, loss=np.inf, thr=np.float32(np.inf))
    if crit == MSE:
        res["counts"] = np.zeros(B, dtype=np.int64)
        res["sums"] = np.zeros((B, 2))
    else:
        res["counts"] = np.zeros((B, K), dtype=np.int64)
    if n == 0:
        return res
    zmin, zmax = z32.min(), z32.max()
    bins = hist_bins(z32, zmin, zmax, B)
    edges = hist_edges(zmin, zmax, B)
    if crit == MSE:
        y = np.asarray(target, dtype=np.float64)
        order = np.argsort(bins, kind="stable")
        yb = y[order]
        cnt = np.bincount(bins, minlength=B).astype(np.int64)
        cuts = np.concatenate([[0], np.cumsum(cnt)])
        s1 = exact_prefix(yb, cuts)
        s2 = exact_prefix(yb, cuts, square=True)
        res["counts"] = cnt
        res["sums"] = np.array([[exact_sum(yb[cuts[b]:cuts[b + 1]]),
                                 exact_sum_sq(yb[cuts[b]:cuts[b + 1]])] for b in range(B)])
        if zmin == zmax:
            return res
        b = np.arange(1, B)
        nL = cuts[b]
        nR = n - nL
        # prefix sums of the left side, each correctly rounded; right = total - left
        # is formed from the exact complement, also correctly rounded.
        s1R = exact_prefix(yb[::-1], n - cuts[b])
        s2R = exact_prefix(yb[::-1], n - cuts[b], square=True)
        loss = mse_children(nL, s1[b], s2[b], nR, s1R, s2R)
    else:
        lab = np.asarray(target, dtype=np.int64)
        counts = np.zeros((B, K), dtype=np.int64)
        np.add.at(counts, (bins, lab), 1)
        res["counts"] = counts
        if zmin == zmax:
            return res
        left = np.cumsum(counts, axis=0)[:-1]     # left[b-1] = bins < b, b = 1..B-1
        right = counts.sum(0)[None, :] - left
        loss = gini_children(left, right) if crit == GINI else entropy_children(left, right)
    if not np.isfinite(loss).any():
        return res
    bi = int(np.argmin(loss))                       # first minimum -> smallest b
    res.update(split=bi + 1, loss=float(loss[bi]), thr=np.float32(edges[bi]))
    return res


def scan_exact(z, target, crit: int, K: int = 0):
    """Exact scan over every boundary between distinct sorted values.

    split = n_L (number of samples sent left) or -1; thr = smallest right value."""
    z = np.asarray(z)
    n = z.size
    res = dict(split=NO_SPLIT, loss=np.inf, thr=np.float32(np.inf))
    if n < 2:
        return res
    order = np.argsort(z, kind="stable")
    zs = z[order]
    cand = np.nonzero(zs[:-1] < zs[1:])[0]          # boundary after sorted position k
    if cand.size == 0:
        return res
    nL = cand + 1
    if crit == MSE:
        ys = np.asarray(target, dtype=np.float64)[order]
        s1L = exact_prefix(ys, nL)
        s2L = exact_prefix(ys, nL, square=True)
        s1R = exact_prefix(ys[::-1], n - nL)
        s2R = exact_prefix(ys[::-1], n - nL, square=True)
        loss = mse_children(nL, s1L, s2L, n - nL, s1R, s2R)
    else:
        lab = np.asarray(target, dtype=np.int64)[order]
        onehot = np.zeros((n, K), dtype=np.int64)
        onehot[np.arange(n), lab] = 1
        pref = np.cumsum(onehot, axis=0)
        left = pref[cand]
        right = pref[-1][None, :] - left
        loss = gini_children(left, right) if crit == GINI else entropy_children(left, right)
    bi = int(np.argmin(loss))
    res.update(split=int(nL[bi]), loss=float(loss[bi]), thr=zs[cand[bi] + 1])
    return res


def split_scan(Z32, target, row_off, P: int, bins: int, crit: int, K: int = 0):
    """Every (node, particle) of a segmented projected matrix Z [N, P].

    Node j owns rows row_off[j]..row_off[j+1]-1; column p of those rows is
    particle p of node j.  bins = 0 selects the exact scan.
    Returns arrays split [nn*P] int64, loss [nn*P] f64, thr [nn*P] f32 and,
    for the histogram scan, counts [nn*P, B, K] (or [nn*P, B]) and sums."""
    Z32 = np.asarray(Z32)
    row_off = np.asarray(row_off, dtype=np.int64)
    nn = row_off.size - 1
    split = np.full(nn * P, NO_SPLIT, dtype=np.int64)
    loss = np.full(nn * P, np.inf)
    thr = np.full(nn * P, np.inf, dtype=np.float32)
    counts, sums = [], []
    for j in range(nn):
        r0, r1 = row_off[j], row_off[j + 1]
        tj = np.asarray(target)[r0:r1]
        for p in range(P):
            zj = Z32[r0:r1, p]
            if bins == 0:
                r = scan_exact(zj, tj, crit, K)
            else:
                r = scan_hist(zj, tj, bins, crit, K)
                counts.append(r["counts"])
                if crit == MSE:
                    sums.append(r["sums"])
            split[j * P + p] = r["split"]
            loss[j * P + p] = r["loss"]
            thr[j * P + p] = r["thr"]
    out = dict(split=split, loss=loss, thr=thr)
    if bins:
        out["counts"] = np.stack(counts) if counts else np.zeros((0,))
        if crit == MSE:
            out["sums"] = np.stack(sums) if sums else np.zeros((0,))
    return out
