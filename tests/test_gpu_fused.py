"""The fused evaluation (projection and histogram scan in one pass, Z never
stored) against the two-kernel path through the C ABI, and the tree built with
it against the tree built without it.  Every projected value is the same
float32 number on both paths, so the bar is bit-exact equality of zmin, zmax,
splits, thresholds and losses (the two-kernel path is itself checked against
the oracle in test_gpu_kernels.py and test_gpu_fullsize.py)."""
import os

import numpy as np
import pytest
import torch

from paper_2208_07023_amd import inputs

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("D,P,sizes,K,bins,crit", [
    (8, 32, [1000], 2, 256, 0),
    (64, 256, [0, 1, 130, 7777, 2], 3, 256, 1),
    (13, 100, [5000, 3, 20000], 4, 64, 0),
    (64, 256, [100000], 3, 256, 1),
    (33, 64, [700] * 64, 2, 7, 1),
    (64, 48, [65000, 70000], 3, 256, 0),
])
def test_fused_equals_two_kernel_path(gpu_lib, D, P, sizes, K, bins, crit):
    api = gpu_lib
    off = inputs.segment_offsets(sizes)
    N, nn = int(off[-1]), len(sizes)
    X, y = inputs.cluster_mixture(N, D, K, seed=D + P)
    W = inputs.random_unit_rows(nn * P, D, seed=P).astype(np.float32)
    Xd, Wd, offd, yd = _t(X), _t(W), _t(off), _t(y)
    f = api.evaluate(Xd, Wd, offd, yd, K, P, bins, crit)
    Z, zmin, zmax = api.project(Xd, Wd, offd, P, tiled=True)
    u = api.split_scan(Z, zmin, zmax, yd, K, offd, P, bins, crit)
    torch.cuda.synchronize()
    assert torch.equal(f["zmin"], zmin) and torch.equal(f["zmax"], zmax)
    assert torch.equal(f["split"], u["split"])
    assert torch.equal(f["thr"], u["thr"])
    assert torch.equal(f["loss"], u["loss"])


def test_fused_tree_equals_two_kernel_tree(gpu_lib):
    api = gpu_lib
    X, y = inputs.cluster_mixture(60000, 32, 3, seed=4, mean_std=0.7)
    cfg = api.TreeConfig(crit=api.ENTROPY, K=3, max_depth=4, min_node=32, P=64, T=6, bins=256,
                         seed=2)
    a = api.grow_tree(_t(X), _t(y), cfg)
    old = os.environ.get("SLM_FUSED")
    os.environ["SLM_FUSED"] = "1"
    try:
        b = api.grow_tree(_t(X), _t(y), cfg)
    finally:
        if old is None:
            del os.environ["SLM_FUSED"]
        else:
            os.environ["SLM_FUSED"] = old
    assert a["n_nodes"] == b["n_nodes"] and a["n_nodes"] > 3
    for k in ("w", "thr", "left", "right", "leaf", "n", "split_loss"):
        assert np.array_equal(a[k], b[k]), k
