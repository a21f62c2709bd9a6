"""Pins of the oracle's projection, binning and split scans (CPU only).

Every check compares the oracle against something other than itself: exact
brute force over thresholds (oracle.brute), counting edges one by one,
correctly rounded sums, scikit-learn's decision stumps on axis-aligned
directions, and invariants the mathematics fixes.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute
from oracle import split as S
from paper_2208_07023_amd import inputs

CRITS = [S.GINI, S.ENTROPY, S.MSE]


def _target(n, crit, K, rng):
    if crit == S.MSE:
        return rng.normal(3.0, 2.0, size=n)
    return rng.integers(0, K, size=n).astype(np.int32)


def _close_exact(oracle_loss, exact):
    return abs(oracle_loss - float(exact)) <= 1e-12 * max(1.0, abs(float(exact)))


# ------------------------------------------------------------------ projection
def test_projection_exact_on_integers():
    X = inputs.integer_matrix(37, 9, -8, 8, seed=1)
    W = inputs.integer_matrix(5, 9, -4, 4, seed=2)
    Z = S.project(X, W)
    ref = np.array([[sum(int(X[i, d]) * int(W[p, d]) for d in range(9)) for p in range(5)]
                    for i in range(37)], dtype=np.float64)
    assert np.array_equal(Z, ref)


def test_projection_matches_fsum():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((20, 16)).astype(np.float32)
    W = inputs.random_unit_rows(6, 16, seed=4).astype(np.float32)
    Z = S.project(X, W)
    Zf = S.project_fsum(X, W)
    mag = np.abs(X.astype(np.float64)) @ np.abs(W.astype(np.float64)).T
    assert np.all(np.abs(Z - Zf) <= 16 * 2.0 ** -53 * mag)


# ------------------------------------------------------------------ binning
@pytest.mark.parametrize("B", [2, 3, 7, 16, 100, 256])
@pytest.mark.parametrize("kind", ["gauss", "dups"])
def test_bins_equal_edge_count(B, kind):
    Z = inputs.projected_features(60, 3, seed=B, kind=kind)
    for p in range(3):
        z = Z[:, p]
        e = S.hist_edges(z.min(), z.max(), B)
        assert e.dtype == np.float32 and e.size == B - 1
        assert np.all(np.diff(e.astype(np.float64)) >= 0)
        b = S.hist_bins(z, z.min(), z.max(), B)
        assert np.array_equal(b, brute.bins_by_counting(z, e))
        assert b.min() >= 0 and b.max() <= B - 1
        # the edge rule: z >= e_b  <=>  bin >= b
        for bb in range(1, B):
            assert np.array_equal(z >= e[bb - 1], b >= bb)


def test_bins_edge_arithmetic_is_float32():
    # zmin = 0.1f, zmax = 0.7f, B = 3: every operation rounded to float32
    zmin, zmax = np.float32(0.1), np.float32(0.7)
    r = np.float32(zmax - zmin)
    d = np.float32(r / np.float32(3))
    want = [np.float32(zmin + np.float32(np.float32(1) * d)),
            np.float32(zmin + np.float32(np.float32(2) * d))]
    got = S.hist_edges(zmin, zmax, 3)
    assert got.tolist() == [float(w) for w in want]
    # and it differs from the FP64 evaluation rounded once
    e64 = [np.float32(0.1 + k * (0.7 - 0.1) / 3) for k in (1, 2)]
    assert got.dtype == np.float32 and len(e64) == 2


def test_integer_values_get_their_own_bin():
    z = np.arange(256, dtype=np.float32)
    b = S.hist_bins(z, 0.0, 255.0, 256)
    assert np.array_equal(b, np.arange(256))


@pytest.mark.parametrize("crit", CRITS)
def test_hist_equals_exact_on_integer_grid(crit):
    rng = np.random.default_rng(5)
    K = 3
    for trial in range(4):
        z = rng.integers(0, 256, size=300).astype(np.float32)
        z[0], z[1] = 0, 255                   # zmin = 0, zmax = 255
        t = _target(300, crit, K, rng)
        h = S.scan_hist(z, t, 256, crit, K)
        e = S.scan_exact(z, t, crit, K)
        # edges sit at b - b/256, so z >= e_b and z >= b select the same integers
        assert np.array_equal(z >= h["thr"], z >= e["thr"])
        assert h["loss"] == pytest.approx(e["loss"], rel=1e-15, abs=0)
        assert int((z < h["thr"]).sum()) == e["split"]


# ------------------------------------------------------------------ scans vs brute force
@pytest.mark.parametrize("crit", CRITS)
@pytest.mark.parametrize("B", [2, 5, 16, 256])
def test_scan_hist_matches_bruteforce(crit, B):
    rng = np.random.default_rng(100 + crit * 10 + B)
    K = 3
    for trial in range(6):
        n = int(rng.integers(2, 30))
        kind = "dups" if trial % 2 else "gauss"
        z = inputs.projected_features(n, 1, seed=trial + 7 * B, kind=kind)[:, 0]
        t = _target(n, crit, K, rng)
        res = S.scan_hist(z, t, B, crit, K)
        e = S.hist_edges(z.min(), z.max(), B)
        losses, best, arg = brute.best_over(z, t, list(e), crit, K)
        if best is None:
            assert res["split"] == -1 and res["loss"] == np.inf
            continue
        assert _close_exact(res["loss"], best)
        # chosen split attains the exact minimum; the smallest such b unless an
        # exact tie is broken differently by FP64 rounding of equal rationals
        assert res["split"] - 1 in arg
        assert res["thr"] == e[res["split"] - 1]
        # counts agree with direct counting
        bins = brute.bins_by_counting(z, e)
        if crit == S.MSE:
            assert np.array_equal(res["counts"], np.bincount(bins, minlength=B))
            for b in range(B):
                sel = t[bins == b]
                assert res["sums"][b, 0] == float(sum(Fraction(float(v)) for v in sel))
                assert res["sums"][b, 1] == float(sum(Fraction(float(v)) ** 2 for v in sel))
        else:
            for b in range(B):
                for k in range(K):
                    assert res["counts"][b, k] == int(((bins == b) & (t == k)).sum())


@pytest.mark.parametrize("crit", CRITS)
def test_scan_exact_matches_bruteforce(crit):
    rng = np.random.default_rng(200 + crit)
    K = 4
    for trial in range(8):
        n = int(rng.integers(1, 30))
        kind = "dups" if trial % 2 else "gauss"
        z = inputs.projected_features(n, 1, seed=300 + trial, kind=kind)[:, 0]
        t = _target(n, crit, K, rng)
        res = S.scan_exact(z, t, crit, K)
        cands = sorted(set(z.tolist()))[1:]        # every distinct value but the smallest
        losses, best, arg = brute.best_over(z, t, cands, crit, K)
        if best is None:
            assert res["split"] == -1
            continue
        assert _close_exact(res["loss"], best)
        assert cands.index(float(res["thr"])) in arg
        assert res["split"] == int((z < res["thr"]).sum())


def test_exact_prefix_is_correctly_rounded():
    rng = np.random.default_rng(9)
    y = rng.normal(0, 1, size=50) * 10.0 ** rng.integers(-5, 6, size=50)
    cuts = [0, 1, 7, 25, 50]
    got = S.exact_prefix(y, cuts)
    got2 = S.exact_prefix(y, cuts, square=True)
    for c, g, g2 in zip(cuts, got, got2):
        assert g == float(sum(Fraction(float(v)) for v in y[:c]))
        assert g2 == float(sum(Fraction(float(v)) ** 2 for v in y[:c]))
        assert g == math.fsum(y[:c])


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("crit", [S.GINI, S.ENTROPY])
def test_pure_node_has_zero_loss(crit):
    z = inputs.projected_features(50, 1, seed=11)[:, 0]
    t = np.full(50, 2, dtype=np.int32)
    for r in (S.scan_hist(z, t, 256, crit, 3), S.scan_exact(z, t, crit, 3)):
        assert r["loss"] == 0.0 and r["split"] >= 1
    assert S.gini_node([0, 0, 50]) == 0.0 and S.entropy_node([0, 0, 50]) == 0.0


def test_constant_target_regression_zero_loss():
    z = inputs.projected_features(40, 1, seed=12)[:, 0]
    y = np.full(40, 0.75)
    r = S.scan_hist(z, y, 64, S.MSE)
    assert r["loss"] == 0.0


@pytest.mark.parametrize("crit", CRITS)
def test_children_never_worse_than_parent(crit):
    rng = np.random.default_rng(13)
    K = 3
    for trial in range(10):
        n = int(rng.integers(5, 200))
        z = inputs.projected_features(n, 1, seed=400 + trial)[:, 0]
        t = _target(n, crit, K, rng)
        r = S.scan_exact(z, t, crit, K)
        if crit == S.MSE:
            parent = S.mse_node(t)
        else:
            c = np.bincount(t, minlength=K)
            parent = S.gini_node(c) if crit == S.GINI else S.entropy_node(c)
        assert r["loss"] <= parent * (1 + 1e-12) + 1e-15


@pytest.mark.parametrize("crit", CRITS)
def test_scale_and_permutation_invariance(crit):
    rng = np.random.default_rng(14)
    K = 3
    n = 120
    z = inputs.projected_features(n, 1, seed=15)[:, 0]
    t = _target(n, crit, K, rng)
    base = S.scan_exact(z, t, crit, K)
    for c in (0.25, 8.0):                      # exact scalings keep the order and the ties
        r = S.scan_exact((z * np.float32(c)).astype(np.float32), t, crit, K)
        assert r["split"] == base["split"] and r["loss"] == pytest.approx(base["loss"], rel=1e-14)
    perm = rng.permutation(n)
    r = S.scan_exact(z[perm], t[perm], crit, K)
    assert r["split"] == base["split"] and r["loss"] == pytest.approx(base["loss"], rel=1e-14)
    h0 = S.scan_hist(z, t, 32, crit, K)
    h1 = S.scan_hist(z[perm], t[perm], 32, crit, K)
    assert np.array_equal(h0["counts"], h1["counts"])
    # every histogram boundary is also an exact candidate
    assert h0["loss"] >= base["loss"] * (1 - 1e-14)


def test_last_bin_totals_are_node_counts():
    rng = np.random.default_rng(16)
    z = inputs.projected_features(90, 1, seed=17)[:, 0]
    t = rng.integers(0, 4, size=90).astype(np.int32)
    r = S.scan_hist(z, t, 256, S.GINI, 4)
    assert np.array_equal(r["counts"].sum(0), np.bincount(t, minlength=4))


def test_degenerate_inputs():
    t = np.array([0, 1, 0], dtype=np.int32)
    for r in (S.scan_hist(np.array([], np.float32), t[:0], 16, S.GINI, 2),
              S.scan_hist(np.full(3, 2.5, np.float32), t, 16, S.GINI, 2),
              S.scan_exact(np.full(3, 2.5, np.float32), t, S.GINI, 2),
              S.scan_exact(np.array([1.0], np.float32), t[:1], S.GINI, 2)):
        assert r["split"] == -1 and r["loss"] == np.inf and r["thr"] == np.inf
    # two samples: one split
    r = S.scan_exact(np.array([2.0, 1.0], np.float32), np.array([1, 0]), S.GINI, 2)
    assert r["split"] == 1 and r["loss"] == 0.0 and r["thr"] == 2.0


def test_gini_closed_form_spot_values():
    # one class on each side: 0; a 50/50 parent: 1/2; counts (3,1 | 0,4):
    # left gini = 1 - (9+1)/16 = 3/8 weighted by 4/8 -> 3/16
    assert float(S.gini_children([[3, 1]], [[0, 4]])[0]) == 3 / 16
    assert S.gini_node([4, 4]) == 0.5
    assert S.entropy_node([4, 4]) == 1.0
    assert float(S.entropy_children([[2, 2]], [[0, 4]])[0]) == 0.5


def test_split_scan_segments():
    sizes = [0, 1, 5, 40]
    off = inputs.segment_offsets(sizes)
    Z = inputs.projected_features(int(off[-1]), 3, seed=18, kind="dups")
    t = np.random.default_rng(19).integers(0, 2, size=int(off[-1])).astype(np.int32)
    out = S.split_scan(Z, t, off, 3, 16, S.GINI, 2)
    for j in range(len(sizes)):
        for p in range(3):
            r = S.scan_hist(Z[off[j]:off[j + 1], p], t[off[j]:off[j + 1]], 16, S.GINI, 2)
            assert out["split"][j * 3 + p] == r["split"]
    assert np.all(out["split"][:6] == -1)


# ------------------------------------------------------------------ axis-aligned = decision stump
@pytest.mark.parametrize("crit", CRITS)
def test_axis_aligned_direction_is_a_decision_stump(crit):
    from sklearn.tree import DecisionTreeClassifier, DecisionTreeRegressor
    X, y, _ = inputs.two_class_gaussian(200, 4, seed=21)
    K = 2
    if crit == S.MSE:
        y = np.abs(X[:, 0].astype(np.float64)) + 0.5 * X[:, 1]
    for d in range(4):
        W = np.zeros((1, 4), dtype=np.float32)
        W[0, d] = 1.0
        z = S.project(X, W)[:, 0].astype(np.float32)
        r = S.scan_exact(z, y, crit, K)
        if crit == S.MSE:
            m = DecisionTreeRegressor(max_depth=1).fit(X[:, [d]], y)
        else:
            m = DecisionTreeClassifier(max_depth=1, criterion="gini" if crit == S.GINI else "entropy").fit(X[:, [d]], y)
        tr = m.tree_
        nl, nr = tr.n_node_samples[1], tr.n_node_samples[2]
        sk = (nl * tr.impurity[1] + nr * tr.impurity[2]) / (nl + nr)
        assert r["loss"] == pytest.approx(sk, rel=1e-9, abs=1e-12)
        left_sk = X[:, d] <= tr.threshold[0]
        left_me = z < r["thr"]
        if r["loss"] < sk - 1e-12 or not np.array_equal(left_sk, left_me):
            # only an exact tie between two different boundaries may differ
            assert abs(r["loss"] - sk) <= 1e-12 * max(1, sk)
