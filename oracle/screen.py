"""Oracle: mixed-precision screening of a swarm evaluation (TEST INFRASTRUCTURE).

The paper evaluates every particle with the same projection (Sec. II-A,
Eq. (1)) and scores it by the loss of its best threshold (Sec. III-B).  For
high-dimensional data it names faster search of the projection as the open
problem (Sec. VI).  This module states one such acceleration as a plain
definition: every particle is first scored on a bfloat16 image of the data and
of its direction, and only the best-scoring few are scored again in float32.

Readings (the paper does not describe this step; these fix it):
* bf16(v) rounds a float32 value to the nearest bfloat16 (8 significand bits,
  ties to even).  The data X is stored in bfloat16.  The screening direction is
  bf16(float32(x)) of the FP64 position x; the re-scoring direction is
  float32(x), the same float32 image the plain evaluation uses.
* The screened projection is the exact dot product of the bfloat16 operands
  rounded to float32 (the GPU accumulates it in float32, so its rounding order
  differs; the parity tests bound that difference).
* Storage of the screened projection (z_bf16): a classification histogram
  search (Gini or entropy, bins > 0) over at most 256 dimensions keeps it in
  bfloat16, the float32 value rounded once more to the nearest bfloat16 (ties
  to even); the scan then reads those values exactly.  It only ranks the
  directions, and the rounding is below the error its bfloat16 operands
  already carry.  Other searches keep float32.
* The re-scored set S holds the k particles with the smallest screened losses,
  ties to the lower index, listed in ascending (loss, index) order.
* The loss handed to the swarm is the re-scored loss for particles of S and
  the screened loss for the others.  Personal bests use that loss; the global
  best only considers particles of S (its loss, split and threshold are those
  of the float32 projection that the tree's partition also uses).
"""
from __future__ import annotations

import numpy as np

from . import split as S


def bf16_round(a):
    """Nearest bfloat16 of float32 values, ties to even, returned as float32.

    A bfloat16 is the upper 16 bits of a binary32.  Rounding adds half an ulp
    of the kept part minus one, plus the lowest kept bit, to the 32-bit pattern
    and clears the low 16 bits; NaNs stay NaNs (quiet)."""
    scalar = np.ndim(a) == 0
    a = np.atleast_1d(np.asarray(a, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    if nan.any():
        q = (u[nan] | np.uint64(0x00400000)) & np.uint64(0xFFFF0000)
        out = out.copy()
        out[nan] = q.astype(np.uint32).view(np.float32)
    return out[0] if scalar else out


def top_k(loss, k: int):
    """Indices of the k smallest losses, ascending by (loss, index)."""
    loss = np.asarray(loss, dtype=np.float64)
    order = np.lexsort((np.arange(loss.size), loss))
    return order[:k]


def screened_storage_bf16(crit: int, bins: int, D: int) -> bool:
    """Whether the screened projection is stored in bfloat16 (see above)."""
    return crit != S.MSE and bins > 0 and D <= 256


def evaluate_screened(Xb, tn, crit: int, K: int, bins: int, k: int, z_bf16=None):
    """Evaluation closure for a swarm with screening.

    Xb: the node's rows as bfloat16 values (float32 array).  The closure takes
    the float32 images W32 [P, D] of the positions and returns
    (loss, split, thr, gloss): the swarm's losses, splits and thresholds and the
    losses eligible for the global best (+inf outside S).  z_bf16: storage of
    the screened projection (None: screened_storage_bf16)."""
    Xb = np.asarray(Xb, dtype=np.float32)
    if z_bf16 is None:
        z_bf16 = screened_storage_bf16(crit, bins, Xb.shape[1])

    def scan_all(Z):
        P = Z.shape[1]
        loss = np.empty(P)
        spl = np.empty(P, dtype=np.int64)
        thr = np.empty(P, dtype=np.float32)
        for p in range(P):
            r = (S.scan_exact(Z[:, p], tn, crit, K) if bins == 0
                 else S.scan_hist(Z[:, p], tn, bins, crit, K))
            loss[p], spl[p], thr[p] = r["loss"], r["split"], r["thr"]
        return loss, spl, thr

    def ev(W32):
        W32 = np.asarray(W32, dtype=np.float32)
        Wb = bf16_round(W32)
        Zs = S.project(Xb, Wb).astype(np.float32)
        loss, spl, thr = scan_all(bf16_round(Zs) if z_bf16 else Zs)
        sel = top_k(loss, min(k, W32.shape[0]))
        lr, sr, tr = scan_all(S.project(Xb, W32[sel]).astype(np.float32))
        loss[sel], spl[sel], thr[sel] = lr, sr, tr
        gloss = np.full(W32.shape[0], np.inf)
        gloss[sel] = lr
        return loss, spl, thr, gloss
    return ev
