"""slm_split_scan_noalloc (the histogram scan with the library's static
per-GPU scratch instead of a caller workspace) against slm_split_scan (a
caller workspace) on the same inputs, through the C ABI: two calls in a row,
the second on a smaller input, every output bit for bit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2208_07023_amd import api, inputs

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _noalloc(Z, zmin, zmax, y, K, off, P, bins, crit):
    lib = api.load()
    nn = off.numel() - 1
    tiled = Z.dim() == 3
    N = Z.shape[1] if tiled else Z.shape[0]
    split = torch.empty(nn * P, dtype=torch.int32, device=Z.device)
    loss = torch.empty(nn * P, dtype=torch.float64, device=Z.device)
    thr = torch.empty(nn * P, dtype=torch.float32, device=Z.device)
    kk = max(K, 1)
    hist = torch.empty(nn * P * bins * kk, dtype=torch.int32, device=Z.device)
    zl = (api.Z_TILED if Z.shape[2] == 32 else api.Z_TILED8) if tiled else api.Z_ROWS
    st = lib.slm_split_scan_noalloc(api._p(Z), zl, api._p(zmin),
                                    api._p(zmax), api._p(y), api.F64 if crit == api.MSE else api.I32,
                                    K, N, api._p(off), nn, P, bins, crit, api._p(split),
                                    api._p(loss), api._p(thr), api._p(hist), None,
                                    api._stream())
    assert st == 0, lib.slm_last_error().decode()
    return dict(split=split, loss=loss, thr=thr, counts=hist.view(nn * P, bins, kk))


@pytest.mark.parametrize("crit", [api.GINI, api.ENTROPY])
def test_noalloc_scan_equals_workspace_scan(gpu_lib, crit):
    K, bins = 3, 256
    cases = [([60_000, 1, 39_999], 256, 11), ([5000, 0, 2500, 700], 64, 12)]
    for sizes, P, seed in cases:   # the second call is smaller than the first
        off = inputs.segment_offsets(sizes)
        N, D = int(off[-1]), 24
        X, y = inputs.cluster_mixture(N, D, K, clusters_per_class=2, mean_std=1.5, seed=seed)
        W = inputs.random_unit_rows(len(sizes) * P, D, seed=seed + 1).astype(np.float32)
        offd = _t(off)
        Z, zmin, zmax = api.project(_t(X), _t(W), offd, P, tiled=True)
        ref = api.split_scan(Z, zmin, zmax, _t(y), K, offd, P, bins, crit, hist=True)
        got = _noalloc(Z, zmin, zmax, _t(y), K, offd, P, bins, crit)
        torch.cuda.synchronize()
        for k in ("split", "loss", "thr", "counts"):
            assert torch.equal(got[k], ref[k]), (sizes, k)
        assert int((ref["split"] > 0).sum()) > 0


def test_noalloc_scan_refuses_what_exceeds_its_scratch(gpu_lib):
    lib = api.load()
    cap = lib.slm_split_scan_noalloc_max_bytes()
    need = lib.slm_split_scan_workspace(4_000_000, 1, 1024, 256, 10, api.GINI)
    assert need > cap
    fake = ctypes.c_void_p(0x1000)
    st = lib.slm_split_scan_noalloc(fake, api.Z_TILED, fake, fake, fake, api.I32, 10, 4_000_000,
                                    fake, 1, 1024, 256, api.GINI, fake, fake, fake, None, None,
                                    None)
    assert st == 4 and b"scratch" in lib.slm_last_error()
    st = lib.slm_split_scan_noalloc(fake, api.Z_TILED, fake, fake, fake, api.I32, 3, 100, fake, 1,
                                    8, 0, api.GINI, fake, fake, fake, None, None, None)
    assert st == 6
