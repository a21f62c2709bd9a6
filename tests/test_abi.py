"""The C ABI library loads, exports every declared entry point and rejects bad
arguments on the host before any launch (CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2208_07023_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slm.h")

pytestmark = pytest.mark.skipif(not os.path.exists(api.LIB_PATH),
                                reason="libslm.so not built (run __graft_entry__.build())")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slm_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(api.LIB_PATH)
    syms = declared_symbols()
    assert {"slm_project", "slm_split_scan", "slm_pso_step", "slm_grow_tree"} <= set(syms)
    for s in syms:
        assert hasattr(lib, s), s
    # and the binding declares a signature for each of them
    assert set(syms) == set(api._SIGS)


def test_version_and_error_strings():
    lib = api.load()
    assert b"gfx950" in lib.slm_version()
    assert lib.slm_last_error() is not None


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation


def _err(lib):
    return lib.slm_last_error().decode()


def test_project_validation():
    lib = api.load()
    st = lib.slm_project(FAKE, api.F32, 10, 0, FAKE, api.F32, FAKE, 1, 4, FAKE, 0, FAKE, FAKE, None)
    assert st == 2 and "D" in _err(lib)
    st = lib.slm_project(FAKE, api.F32, 10, 4, FAKE, api.BF16, FAKE, 1, 4, FAKE, 0, FAKE, FAKE, None)
    assert st == 3
    st = lib.slm_project(FAKE, api.F32, 10, 4, FAKE, api.F32, FAKE, 1, 0, FAKE, 0, FAKE, FAKE, None)
    assert st == 2
    st = lib.slm_project(None, api.F32, 10, 4, FAKE, api.F32, FAKE, 1, 4, FAKE, 0, FAKE, FAKE, None)
    assert st == 1 and "NULL" in _err(lib)
    st = lib.slm_project(FAKE, api.F32, 10, 4, FAKE, api.F32, FAKE, 1, 4, FAKE, 4, FAKE, FAKE, None)
    assert st == 1 and "layout" in _err(lib)
    # 8-particle tiles: 96 N + 32 * 65600 + 124 bytes must stay below 2^31
    # (the first N refused, as the header states); bfloat16 tiles double it
    for zl, n in ((api.Z_TILED8, 22_347_754), (api.Z_TILED8_BF16, 44_717_375)):
        st = lib.slm_project(FAKE, api.F32, n, 4, FAKE, api.F32, FAKE, 1, 4, FAKE,
                             zl, FAKE, FAKE, None)
        assert st == 1 and "TILED8" in _err(lib)
    # nothing to do: returns OK without touching the device
    st = lib.slm_project(None, api.F32, 0, 4, None, api.F32, None, 0, 4, None, 0, None, None, None)
    assert st == 0


def test_split_scan_validation():
    lib = api.load()
    args = lambda **kw: dict(dict(Z=FAKE, zl=api.Z_ROWS, zmin=FAKE, zmax=FAKE, t=FAKE, tt=api.I32, K=3, N=100,
                                  off=FAKE, nn=1, P=8, bins=16, crit=api.GINI, ws=FAKE,
                                  wsb=1 << 30), **kw)

    def call(a):
        return lib.slm_split_scan(a["Z"], a["zl"], a["zmin"], a["zmax"], a["t"], a["tt"], a["K"], a["N"],
                                  a["off"], a["nn"], a["P"], a["bins"], a["crit"], FAKE, FAKE,
                                  FAKE, None, None, a["ws"], a["wsb"], None)
    assert call(args(bins=1)) == 2
    assert call(args(bins=257)) == 2
    assert call(args(K=1)) == 2
    assert call(args(K=17)) == 2
    assert call(args(crit=3)) == 1
    assert call(args(tt=api.F64)) == 3                      # classification needs I32
    assert call(args(crit=api.MSE, tt=api.I32, K=0)) == 3   # MSE needs F64
    assert call(args(crit=api.MSE, tt=api.F64, K=3)) == 2
    assert call(args(wsb=16)) == 4 and "workspace" in _err(lib)
    assert call(args(zmin=None)) == 1
    assert call(args(zl=4)) == 1 and "layout" in _err(lib)
    assert call(args(zl=api.Z_TILED8, N=22_347_754)) == 1 and "TILED8" in _err(lib)
    assert call(args(zl=api.Z_TILED8_BF16, N=44_717_375)) == 1 and "TILED8" in _err(lib)
    # bfloat16 Z: classification histogram scans only
    assert call(args(zl=api.Z_TILED8_BF16, crit=api.MSE, tt=api.F64, K=0)) == 6
    assert call(args(zl=api.Z_TILED8_BF16, bins=0)) == 6 and "bfloat16" in _err(lib)
    need = lib.slm_split_scan_workspace(100, 1, 8, 16, 3, api.GINI)
    assert need > 0
    assert lib.slm_split_scan_workspace(4_000_000, 2048, 1024, 256, 10, api.GINI) < 8 << 30


def test_pso_validation():
    lib = api.load()
    st = lib.slm_pso_init(*([FAKE] * 7), FAKE, 1, 8, 5000, 1, 0, FAKE, api.F32, None)
    assert st == 2
    st = lib.slm_pso_init(*([FAKE] * 7), FAKE, 1, 8, 4, 1, 0, FAKE, api.F64, None)
    assert st == 3
    # loss, gloss, split, thr, gbest_split, gbest_thr: split given without gbest_split
    st = lib.slm_pso_step(*([FAKE] * 7), FAKE, None, FAKE, None, None, None, FAKE, 1, 8, 4,
                          0.7, 1.5, 1.5, 1, 0, 1, 1, FAKE, api.F32, None)
    assert st == 1
    st = lib.slm_pso_step(*([FAKE] * 7), FAKE, None, None, None, None, None, FAKE, 1, 8, 4,
                          float("nan"), 1.5, 1.5, 1, 0, 1, 1, FAKE, api.F32, None)
    assert st == 1


def test_screen_validation():
    lib = api.load()
    assert lib.slm_screen_select(FAKE, 2, 8, 9, FAKE, None) == 2          # k > P
    assert lib.slm_screen_select(FAKE, 2, 8, 0, FAKE, None) == 2          # k = 0
    assert lib.slm_screen_select(None, 2, 8, 4, FAKE, None) == 1
    assert lib.slm_screen_select(None, 0, 8, 4, None, None) == 0          # nothing to do
    assert lib.slm_screen_gather(FAKE, FAKE, 2, 8, 4, 0, FAKE, None) == 2  # D = 0
    assert lib.slm_screen_gather(FAKE, None, 2, 8, 4, 3, FAKE, None) == 1
    assert lib.slm_screen_merge(FAKE, FAKE, FAKE, FAKE, 2, 8, 16, FAKE, FAKE, FAKE, FAKE,
                                None) == 2
    assert lib.slm_screen_merge(FAKE, FAKE, FAKE, FAKE, 2, 8, 4, FAKE, FAKE, FAKE, None,
                                None) == 1
    # the mixed projection takes (BF16, F32); (F32, BF16) is refused
    st = lib.slm_project(None, api.BF16, 0, 4, None, api.F32, None, 0, 4, None, 0, None, None, None)
    assert st == 0


def test_evaluate_validation():
    lib = api.load()
    args = lambda D=8, K=3, bins=64, crit=api.GINI: (FAKE, 100, D, FAKE, FAKE, 1, 8, FAKE, K, bins,
                                                     crit, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE,
                                                     1 << 30, None)
    assert lib.slm_evaluate(*args(D=65)) == 6
    assert lib.slm_evaluate(*args(K=5)) == 6
    assert lib.slm_evaluate(*args(crit=api.MSE)) == 6
    assert lib.slm_evaluate(*args(bins=1)) == 2
    a = list(args())
    a[17] = 16
    assert lib.slm_evaluate(*a) == 4


def test_grow_tree_precision_validation():
    lib = api.load()
    out = api.TreeOut()
    for kw, want in ((dict(precision=2), 1), (dict(precision=1, rescore_k=0), 2),
                     (dict(precision=1, rescore_k=9), 2)):
        cfg = api.TreeConfig(crit=api.GINI, K=2, P=8, T=2, bins=16, **kw)
        prm = cfg.c_params()
        assert lib.slm_grow_tree_workspace(ctypes.byref(prm), 1000, 8) == 0
        st = lib.slm_grow_tree(FAKE, api.BF16, 1000, 8, FAKE, api.I32, ctypes.byref(prm), FAKE,
                               1 << 30, ctypes.byref(out), None)
        assert st == want, kw
    cfg = api.TreeConfig(crit=api.GINI, K=2, P=8, T=2, bins=16, precision=1, rescore_k=4)
    prm = cfg.c_params()
    plain = api.TreeConfig(crit=api.GINI, K=2, P=8, T=2, bins=16).c_params()
    # screening needs room for the re-scored projection; bfloat16 rows halve X
    assert lib.slm_grow_tree_workspace(ctypes.byref(prm), 1000, 8) > 0
    st = lib.slm_grow_tree(FAKE, api.F32, 1000, 8, FAKE, api.I32, ctypes.byref(prm), FAKE,
                           1 << 30, ctypes.byref(out), None)
    assert st == 3 and "BF16" in _err(lib)
    del plain


def test_grow_tree_params_validation():
    lib = api.load()
    ok = api.TreeConfig(crit=api.ENTROPY, K=3, max_depth=8, P=256, T=50, bins=256).c_params()
    assert lib.slm_grow_tree_workspace(ctypes.byref(ok), 100_000, 64) > 100_000 * 256 * 4
    for bad in (dict(K=1), dict(bins=1), dict(P=0), dict(crit=api.MSE, K=3), dict(min_node=0)):
        cfg = api.TreeConfig(crit=api.ENTROPY, K=3, P=8, T=2, bins=16)
        for k, v in bad.items():
            setattr(cfg, k, v)
        prm = cfg.c_params()
        assert lib.slm_grow_tree_workspace(ctypes.byref(prm), 1000, 8) == 0
        out = api.TreeOut()
        st = lib.slm_grow_tree(FAKE, api.F32, 1000, 8, FAKE, api.I32, ctypes.byref(prm), FAKE,
                               1 << 30, ctypes.byref(out), None)
        assert st in (1, 2), bad
        assert _err(lib)


def test_binding_refuses_host_tensors():
    import torch
    with pytest.raises(TypeError):
        api.project(torch.zeros(4, 2), torch.zeros(1, 2), torch.tensor([0, 4]), 1)


def test_dft_validation():
    lib = api.load()
    args = lambda D=8, n=3, K=3, bins=64, crit=api.GINI, tt=api.I32: (
        FAKE, 100, D, FAKE, 2, FAKE, tt, K, bins, crit, n, FAKE, FAKE, FAKE, 1 << 30, None)
    assert lib.slm_dft_select(*args(n=0)) == 2
    assert lib.slm_dft_select(*args(n=9)) == 2
    assert lib.slm_dft_select(*args(D=5000, n=3)) == 2
    assert lib.slm_dft_select(*args(crit=3)) == 1
    assert lib.slm_dft_select(*args(bins=1)) == 2
    assert lib.slm_dft_select(*args(K=1)) == 3
    assert lib.slm_dft_select(*args(crit=api.MSE, K=0, tt=api.I32)) == 3
    assert lib.slm_dft_select_workspace(100, 8, 2, 64, 3, api.GINI) > 256
    sub = lambda sel, n_sel: lib.slm_pso_init_subspace(*([FAKE] * 8), 2, 8, 6, 0, 0, FAKE, api.F32,
                                                       sel, n_sel, None)
    assert sub(None, 3) == 1
    assert sub(FAKE, 0) == 2
    assert sub(FAKE, 7) == 2


def test_grow_tree_dft_validation():
    lib = api.load()
    out = api.TreeOut()
    for kw, want in ((dict(dft_top_n=9), 2), (dict(dft_top_n=-1), 2),
                     (dict(dft_top_n=3, precision=1, rescore_k=4), 6)):
        cfg = api.TreeConfig(crit=api.GINI, K=2, P=8, T=2, bins=16, **kw)
        prm = cfg.c_params()
        assert lib.slm_grow_tree_workspace(ctypes.byref(prm), 1000, 8) == 0
        xt = api.BF16 if kw.get("precision") == 1 else api.F32
        st = lib.slm_grow_tree(FAKE, xt, 1000, 8, FAKE, api.I32, ctypes.byref(prm), FAKE,
                               1 << 30, ctypes.byref(out), None)
        assert st == want, kw
    for n in (0, 3, 8):   # accepted: off, a subspace, all dimensions
        prm = api.TreeConfig(crit=api.GINI, K=2, P=8, T=2, bins=16, dft_top_n=n).c_params()
        assert lib.slm_grow_tree_workspace(ctypes.byref(prm), 1000, 8) > 0


def test_probabilistic_search_validation():
    lib = api.load()
    cand = lambda R, ranks=FAKE: lib.slm_ps_candidates(FAKE, FAKE, api.F32, FAKE, 2, 8, 6, ranks,
                                                       R, FAKE, FAKE, 0, 0, 0, None)
    assert cand(0) == 2 and cand(7) == 2 and cand(65) == 2
    assert cand(3, ranks=None) == 1
    prm = api.TreeConfig(crit=api.GINI, K=2, P=8, T=2, bins=16).c_params()
    prm.proposal = 2
    for R, pd, want_ok in ((0, FAKE, False), (9, FAKE, False), (3, None, False), (3, FAKE, True)):
        prm.ps_R, prm.ps_pd, prm.ps_amax = R, pd, FAKE
        assert (lib.slm_grow_tree_workspace(ctypes.byref(prm), 1000, 8) > 0) == want_ok, R
    prm.ps_R, prm.ps_pd, prm.dft_top_n = 3, FAKE, 4
    assert lib.slm_grow_tree_workspace(ctypes.byref(prm), 1000, 8) == 0


def test_forest_and_boost_validation():
    lib = api.load()
    out = api.TreeOut()
    prm = api.TreeConfig(crit=api.GINI, K=3, max_depth=4, P=8, T=2, bins=16).c_params()
    one = lib.slm_grow_tree_workspace(ctypes.byref(prm), 1000, 8)
    four = lib.slm_grow_forest_workspace(ctypes.byref(prm), 1000, 8, 4)
    # four trees: four gathered copies of the rows ahead of a 4000-row tree workspace
    assert four > 4 * 1000 * 8 * 4 + lib.slm_grow_tree_workspace(ctypes.byref(prm), 4000, 8) - 4096
    assert four > 3 * one
    for nt in (0, 70000):
        assert lib.slm_grow_forest_workspace(ctypes.byref(prm), 1000, 8, nt) == 0
        st = lib.slm_grow_forest(FAKE, api.F32, 1000, 8, FAKE, api.I32, ctypes.byref(prm), nt, 1,
                                 FAKE, 1 << 40, None, ctypes.byref(out), None, None)
        assert st == 2 and "n_trees" in _err(lib)
    # n_trees * N must stay below 2^31
    assert lib.slm_grow_forest_workspace(ctypes.byref(prm), 1 << 20, 8, 4096) == 0
    st = lib.slm_grow_forest(FAKE, api.F32, 1000, 8, FAKE, api.I32, ctypes.byref(prm), 2, 2, FAKE,
                             1 << 40, None, ctypes.byref(out), None, None)
    assert st == 1   # NULL output arrays are found before the bootstrap flag
    pred = lambda K, nt=2: lib.slm_forest_predict(FAKE, FAKE, FAKE, FAKE, FAKE, 5, FAKE, nt, 8, K,
                                                  FAKE, 10, FAKE, FAKE, None)
    assert pred(1) == 2 and pred(17) == 2 and pred(3, nt=0) == 2
    # boosting grows SLR trees: an MSE parameter set with K = 0
    mse = api.TreeConfig(crit=api.MSE, K=0, max_depth=3, P=8, T=2, bins=16).c_params()
    assert lib.slm_boost_workspace(ctypes.byref(mse), 1000, 8, 0) > 0
    assert lib.slm_boost_workspace(ctypes.byref(mse), 1000, 8, 3) > \
        lib.slm_boost_workspace(ctypes.byref(mse), 1000, 8, 0)
    assert lib.slm_boost_workspace(ctypes.byref(prm), 1000, 8, 3) == 0
    assert lib.slm_boost_workspace(ctypes.byref(mse), 1000, 8, 1) == 0
    assert lib.slm_boost_workspace(ctypes.byref(mse), 1000, 8, 17) == 0
    st = lib.slm_boost(FAKE, 1000, 8, FAKE, api.F64, 3, ctypes.byref(mse), 2, 0.1, FAKE, 1 << 40,
                       FAKE, FAKE, ctypes.byref(out), None, None)
    assert st == 3 and "labels" in _err(lib)
    st = lib.slm_boost(FAKE, 1000, 8, FAKE, api.F64, 0, ctypes.byref(mse), 2, float("nan"), FAKE,
                       1 << 40, FAKE, FAKE, ctypes.byref(out), None, None)
    assert st == 1 and "lr" in _err(lib)


def test_exact_scan_tree_refuses_large_roots():
    """The exact scan (bins = 0) sorts a node in one work-group's LDS, at most
    8192 rows; a tree, forest or boosting round whose root holds more rows is
    refused before any launch (Sec. II-A, Eqs. (3)-(4) are not silently
    replaced by a leaf)."""
    lib = api.load()
    out = api.TreeOut()
    cls = api.TreeConfig(crit=api.GINI, K=2, max_depth=3, P=8, T=2, bins=0).c_params()
    assert lib.slm_grow_tree_workspace(ctypes.byref(cls), 8192, 8) > 0
    assert lib.slm_grow_tree_workspace(ctypes.byref(cls), 8193, 8) == 0
    st = lib.slm_grow_tree(FAKE, api.F32, 8193, 8, FAKE, api.I32, ctypes.byref(cls), FAKE,
                           1 << 40, ctypes.byref(out), None)
    assert st == 6 and "8192" in _err(lib)
    assert lib.slm_grow_forest_workspace(ctypes.byref(cls), 8192, 8, 3) > 0
    assert lib.slm_grow_forest_workspace(ctypes.byref(cls), 10_000, 8, 3) == 0
    st = lib.slm_grow_forest(FAKE, api.F32, 10_000, 8, FAKE, api.I32, ctypes.byref(cls), 3, 1,
                             FAKE, 1 << 40, None, ctypes.byref(out), None, None)
    assert st == 6 and "8192" in _err(lib)
    mse = api.TreeConfig(crit=api.MSE, K=0, max_depth=3, P=8, T=2, bins=0).c_params()
    assert lib.slm_boost_workspace(ctypes.byref(mse), 8192, 8, 0) > 0
    assert lib.slm_boost_workspace(ctypes.byref(mse), 8193, 8, 0) == 0
    st = lib.slm_boost(FAKE, 8193, 8, FAKE, api.F64, 0, ctypes.byref(mse), 2, 0.1, FAKE, 1 << 40,
                       FAKE, FAKE, ctypes.byref(out), None, None)
    assert st == 6 and "8192" in _err(lib)
    # the histogram scan has no such limit
    hist = api.TreeConfig(crit=api.GINI, K=2, max_depth=3, P=8, T=2, bins=16).c_params()
    assert lib.slm_grow_tree_workspace(ctypes.byref(hist), 1 << 20, 8) > 0


def test_tables_and_boost_scores_validation():
    lib = api.load()
    assert lib.slm_ps_tables(0, 10.0, FAKE, FAKE, None) == 2
    assert lib.slm_ps_tables(65, 10.0, FAKE, FAKE, None) == 2
    assert lib.slm_ps_tables(8, 0.5, FAKE, FAKE, None) == 1
    assert lib.slm_ps_tables(8, float("inf"), FAKE, FAKE, None) == 1
    assert lib.slm_ps_tables(8, 10.0, None, FAKE, None) == 1
    import numpy as np
    f0 = np.zeros(3)
    bs = lambda nr, nc, lr=0.1, F=FAKE: lib.slm_boost_scores(
        FAKE, FAKE, FAKE, FAKE, FAKE, 7, FAKE, nr, nc, 8, f0.ctypes.data, lr, FAKE, 100, FAKE, F,
        None)
    assert bs(2, 1) == 2 and bs(2, 17) == 2 and bs(-1, 0) == 2
    assert bs(2, 3, lr=float("nan")) == 1
    assert bs(2, 3, F=None) == 1


def test_autotune_validation(tmp_path):
    lib = api.load()
    assert lib.slm_autotune_set(3, None) == 1
    assert lib.slm_autotune_set(-1, None) == 1
    assert lib.slm_autotune_set(2, None) == 1 and "file" in _err(lib)
    # a plans file is read back (malformed entries are skipped)
    p = tmp_path / "plans.json"
    p.write_text('{"plans": {"scan/x/N1/n1/P1/B2/K2/c0": [8, 4096], "proj/x/k3/D8/P1/N1": [1, 0]}}')
    assert lib.slm_autotune_set(1, str(p).encode()) == 0
    assert lib.slm_autotune_plans() == 2
    assert lib.slm_autotune_set(0, None) == 0
    assert lib.slm_autotune_set(1, None) == 0   # back to the default
