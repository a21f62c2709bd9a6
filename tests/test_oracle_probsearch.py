"""Pins of the probabilistic-search oracle (Sec. II-B): table shape, the
candidates' support, range and norm, the selection and value frequencies
against the stated probabilities, the R = 1 special case, and that the search
returns the minimum over everything it evaluated."""
import numpy as np
import pytest

from oracle import probsearch as PS
from oracle import split as S


def test_tables():
    pd, am = PS.tables(8, 10.0)
    assert pd[0] == 1.0 and am[0] == 10 and am[-1] == 1
    assert np.all(np.diff(pd) < 0) and np.all(np.diff(am) <= 0)
    pd1, am1 = PS.tables(1, 6.0)
    assert pd1[0] == 1.0 and am1[0] == 6


def test_candidates_support_range_and_norm():
    D, R, P = 20, 6, 300
    ranks = np.random.default_rng(0).permutation(D)
    pd, am = PS.tables(R, 8.0)
    coef, rk = PS.coefficients(3, 1, 9, 4, P, ranks, pd, am)
    assert np.array_equal(rk, ranks[:R])
    assert np.all(np.abs(coef) <= am[None, :]) and np.all((coef != 0).any(axis=1))
    x = PS.candidates(3, 1, 9, 4, P, D, ranks, pd, am)
    out = np.setdiff1d(np.arange(D), ranks[:R])
    assert np.all(x[:, out] == 0.0)
    assert np.allclose(np.linalg.norm(x, axis=1), 1.0, rtol=0, atol=4e-16)
    # the direction is the integer vector scaled: ratios are exact integer ratios
    c0 = coef[0]
    nz = np.nonzero(c0)[0][0]
    assert np.allclose(x[0, ranks[:R]] / x[0, ranks[nz]], c0 / c0[nz], rtol=0, atol=1e-15)


def test_selection_and_value_frequencies():
    R, P = 5, 6000
    pd, am = PS.tables(R, 4.0)
    coef, _ = PS.coefficients(11, 0, 2, 1, P, np.arange(R), pd, am)
    for d in range(R):
        used = coef[:, d] != 0
        # rank 1 also takes +1 when nothing else is selected
        p_exp = pd[d] if d else 1.0
        sd = np.sqrt(p_exp * (1 - p_exp) / P) + 1e-12
        if d:
            assert abs(used.mean() - p_exp) <= 4 * sd + 1e-3, d
        vals = coef[used, d]
        m = am[d]
        for v in list(range(1, m + 1)) + list(range(-m, 0)):
            f = np.mean(vals == v)
            assert abs(f - 1 / (2 * m)) <= 4 * np.sqrt((1 / (2 * m)) / len(vals)) + 0.01, (d, v)


def test_single_rank_gives_signed_unit_vectors():
    pd, am = PS.tables(1, 5.0)
    x = PS.candidates(5, 0, 1, 0, 64, 7, [3, 0, 1], pd, am)
    assert np.all(np.abs(x[:, 3]) == 1.0) and np.all(np.delete(x, 3, axis=1) == 0.0)


def test_search_returns_the_minimum_over_all_candidates():
    rng = np.random.default_rng(4)
    n, D, K = 200, 6, 2
    y = rng.integers(0, K, n).astype(np.int32)
    X = (rng.normal(0, 1, (n, D)) + y[:, None] * rng.normal(0, 1, D)).astype(np.float32)
    ranks = np.arange(D)
    pd, am = PS.tables(4, 6.0)
    seen = []

    def ev(W32):
        Z = S.project(X, W32).astype(np.float32)
        out = [S.scan_hist(Z[:, p], y, 32, S.GINI, K) for p in range(W32.shape[0])]
        loss = np.array([o["loss"] for o in out])
        seen.extend(loss.tolist())
        return (loss, np.array([o["split"] for o in out]), np.array([o["thr"] for o in out]))

    res = PS.run_search(ev, 8, D, 5, 2, 0, 0, ranks, pd, am)
    assert res["loss"] == min(seen)
    assert np.all(np.diff(res["history"]) <= 0) and res["evals"] == 6


def test_tree_with_probabilistic_search_splits_on_ranked_channels():
    from oracle import dft, tree as OT
    rng = np.random.default_rng(6)
    n, D, K = 300, 8, 2
    y = rng.integers(0, K, n).astype(np.int32)
    X = (rng.normal(0, 1, (n, D)) + 2.0 * y[:, None] * (np.arange(D) < 3)).astype(np.float32)
    prm = OT.TreeParams(crit=S.GINI, K=K, max_depth=1, min_node=10, P=8, T=4, bins=32, seed=3,
                        search=2, ps_R=3, ps_alpha0=4.0)
    tr = OT.grow_tree(X, y, prm).arrays()
    top = dft.top_n(dft.dft_losses(X, y, S.GINI, K, 32), 3)
    assert set(np.nonzero(tr["w"][0])[0].tolist()) <= set(top.tolist())
    assert tr["split_loss"][0] < tr["impurity"][0]
