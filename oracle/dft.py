"""Oracle: the discriminant feature test (DFT) of a node and its top-n channel
selection (Alg. 2: run the DFT for the node, select its top n channels, run
the swarm in those n dimensions).  Test infrastructure only.

Readings of the paper used here (Sec. II-A names the DFT as the test that
picks the threshold of a 1-D subspace; Alg. 2 re-computes the top n
discriminant features of every node as the swarm's input dimensions):
* the DFT loss of input feature d is the loss of its best threshold, scanned
  exactly as any projected feature is: x_d is the projection on the unit
  vector e_d, binned with the float32 edges over the node's [min, max] of x_d
  (histogram scan) or split at every boundary between distinct values (exact
  scan), under the tree's criterion;
* the top n channels are the n features of smallest DFT loss, ties to the
  lower index; a feature without a valid split (loss +inf) sorts last;
* the swarm runs in the span of the selected unit vectors: its start draws
  the same N(0, I) numbers as the full start (oracle.pso.init_positions),
  zeroes the coordinates of the unselected features and scales each row to
  unit norm.  The moves keep those coordinates at zero, since x, v, the
  personal bests and the global best are all zero there.
"""
from __future__ import annotations

import numpy as np

from . import screen
from . import split as S
from .pso import init_positions


def dft_losses(Xn, tn, crit: int, K: int, bins: int):
    """DFT loss [D] of every input feature of one node (rows Xn, targets tn)."""
    Xf = np.asarray(Xn, dtype=np.float32)
    loss = np.empty(Xf.shape[1])
    for d in range(Xf.shape[1]):
        z = Xf[:, d]
        r = S.scan_exact(z, tn, crit, K) if bins == 0 else S.scan_hist(z, tn, bins, crit, K)
        loss[d] = r["loss"]
    return loss


def top_n(loss, n: int):
    """The n channels of smallest DFT loss, ascending by (loss, index)."""
    return screen.top_k(loss, n)


def subspace_start(seed, tree, node, P, D, sel):
    """Initial positions [P, D] restricted to the channels `sel`."""
    mask = np.zeros(D, dtype=bool)
    mask[np.asarray(sel, dtype=np.int64)] = True
    return init_positions(seed, tree, node, P, D, mask=mask)
