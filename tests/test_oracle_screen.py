"""Pins of the oracle's bfloat16 screening with float32 re-scoring (CPU only).

Each pin checks the oracle against something other than its own formula: the
bfloat16 rounding against hand-worked values and torch's CPU conversion, the
selection against its defining properties, the screened evaluation against the
plain float32 evaluation in the cases where the two must coincide, and the
swarm's global-best rule against a planted case."""
import numpy as np
import pytest
import torch

from oracle import pso as O
from oracle import screen as SC
from oracle import split as S
from oracle import tree as TR
from paper_2208_07023_amd import inputs


# ------------------------------------------------------------------ bf16
def test_bf16_round_hand_values():
    # bf16 keeps 8 significand bits: the ulp of [1, 2) is 2^-7
    cases = {
        1.0: 1.0,
        1.0 + 2.0 ** -8: 1.0,                           # tie -> even (mantissa 0)
        1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,           # tie -> even (mantissa 2)
        1.0 + 2.0 ** -8 + 2.0 ** -20: 1.0 + 2.0 ** -7,  # above the tie -> up
        -(1.0 + 2.0 ** -8): -1.0,
        0.0: 0.0,
        2.0 ** -130: 2.0 ** -130,                       # subnormal, exact in bf16
    }
    for v, want in cases.items():
        got = float(SC.bf16_round(np.float32(v)))
        assert got == np.float32(want), (v, got, want)
    # halfway between the largest finite bfloat16 (odd significand) and
    # infinity: ties to even gives infinity; just below it stays finite
    tie = np.array([0x7F7F8000, 0x7F7F7FFF], dtype=np.uint32).view(np.float32)
    r = SC.bf16_round(tie)
    assert np.isinf(r[0]) and r[1].view(np.uint32) == 0x7F7F0000
    assert np.isnan(SC.bf16_round(np.float32(np.nan)))
    assert str(SC.bf16_round(np.float32(-0.0))) == "-0.0"


def test_bf16_round_matches_torch_cpu_conversion():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        rng.integers(-300, 300, 5000) + 0.5,
                        (1 + np.arange(1, 128) * 2.0 ** -8)]).astype(np.float32)
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    got = SC.bf16_round(a)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_bf16_round_agrees_with_storage_rounding_of_the_inputs():
    rng = np.random.default_rng(1)
    a = (rng.standard_normal(4096) * 3).astype(np.float32)
    stored = inputs.bf16_bits_to_f32(inputs.f32_to_bf16_bits(a))
    assert np.array_equal(SC.bf16_round(a), stored)


# ------------------------------------------------------------------ selection
@pytest.mark.parametrize("P,k,ties", [(32, 8, False), (64, 32, True), (7, 7, True), (300, 32, True)])
def test_top_k_defining_properties(P, k, ties):
    rng = np.random.default_rng(P + k)
    loss = (rng.integers(0, 5, P) / 4.0) if ties else rng.uniform(0, 1, P)
    loss[rng.integers(0, P, 3)] = np.inf
    sel = SC.top_k(loss, k)
    assert len(sel) == k and len(set(sel.tolist())) == k
    rest = np.setdiff1d(np.arange(P), sel)
    if rest.size:
        assert loss[sel].max() <= loss[rest].min()
        # at the boundary value the lower indices are the selected ones
        edge = loss[sel].max()
        assert sel[loss[sel] == edge].max() < rest[loss[rest] == edge].min(initial=P)
    # listed in ascending (loss, index) order
    pairs = list(zip(loss[sel], sel))
    assert all(pairs[i] < pairs[i + 1] for i in range(k - 1))


def test_top_k_brute_force_tiny():
    rng = np.random.default_rng(5)
    for _ in range(200):
        P = int(rng.integers(1, 9))
        k = int(rng.integers(1, P + 1))
        loss = rng.integers(0, 3, P) / 2.0
        # brute force: repeatedly take the first index holding the minimum
        left, want = list(range(P)), []
        for _ in range(k):
            m = min(loss[i] for i in left)
            i = next(i for i in left if loss[i] == m)
            want.append(i)
            left.remove(i)
        assert SC.top_k(loss, k).tolist() == want


# ------------------------------------------------------------------ screened evaluation
def _plain_eval(Xb, tn, crit, K, bins):
    return TR.evaluate_node(Xb, tn, TR.TreeParams(crit=crit, K=K, bins=bins))


@pytest.mark.parametrize("crit,K,bins", [(S.GINI, 3, 64), (S.ENTROPY, 2, 0), (S.MSE, 0, 32)])
def test_screen_with_k_equal_P_is_the_plain_evaluation(crit, K, bins):
    """Re-scoring every particle leaves nothing of the screen in the result."""
    rng = np.random.default_rng(7)
    n, D, P = 300, 12, 16
    Xb = SC.bf16_round(rng.standard_normal((n, D)).astype(np.float32))
    tn = rng.standard_normal(n) if crit == S.MSE else rng.integers(0, K, n)
    W32 = inputs.random_unit_rows(P, D, seed=8).astype(np.float32)
    l0, s0, t0 = _plain_eval(Xb, tn, crit, K, bins)(W32)
    l1, s1, t1, g1 = SC.evaluate_screened(Xb, tn, crit, K, bins, P)(W32)
    assert np.array_equal(l0, l1) and np.array_equal(s0, s1) and np.array_equal(t0, t1)
    assert np.array_equal(g1, l1)


def test_screened_storage_rounds_to_bfloat16_hand_case():
    """Storage of the screened projection, by hand.  Rows x = (1, 0), (1, 1),
    (1, 2), labels 0, 1, 1; particle 0 is w = (1, 2^-8) (a bfloat16 value),
    so its exact projections are 1, 1 + 2^-8, 1 + 2^-7.  With 4 bins the
    float32 edges are 1 + j 2^-9, the bins 0, 2, 3 and the labels separate
    (Gini 0).  Stored in bfloat16, 1 + 2^-8 is a tie between 1 and 1 + 2^-7
    and goes to the even 1: bins 0, 0, 3, best split {0, 1} | {1} with Gini
    (2/3) (1/2) = 1/3.  Particle 1, w = (0, 1), projects to 0, 1, 2 and
    separates in either storage, so it is the re-scored top 1 and particle 0
    keeps its screened loss."""
    Xb = np.array([[1, 0], [1, 1], [1, 2]], np.float32)
    tn = np.array([0, 1, 1])
    W32 = np.array([[1, 2.0 ** -8], [0, 1]], np.float32)
    assert np.array_equal(SC.bf16_round(W32), W32) and SC.screened_storage_bf16(S.GINI, 4, 2)
    l, s, t, g = SC.evaluate_screened(Xb, tn, S.GINI, 2, 4, 1)(W32)
    assert l[0] == pytest.approx(1.0 / 3.0, abs=1e-15) and l[1] == 0.0
    assert np.isinf(g[0]) and g[1] == 0.0
    l32, _, _, g32 = SC.evaluate_screened(Xb, tn, S.GINI, 2, 4, 1, z_bf16=False)(W32)
    assert l32[0] == 0.0 and l32[1] == 0.0 and g32[0] == 0.0   # tie: the lower index re-scored
    # regression and the exact scan keep float32 storage
    assert not SC.screened_storage_bf16(S.MSE, 4, 2) and not SC.screened_storage_bf16(S.GINI, 0, 2)
    assert not SC.screened_storage_bf16(S.GINI, 4, 257)


def test_screen_is_exact_when_directions_are_bf16_values():
    """Data and directions already representable in bfloat16, float32
    storage of the screened projection: both projections are the same
    float32 numbers, so the screened loss of every particle equals its
    re-scored loss and the plain loss."""
    rng = np.random.default_rng(9)
    n, D, P, k = 400, 10, 24, 5
    Xb = (rng.integers(-16, 17, (n, D)) / 4.0).astype(np.float32)
    W32 = (rng.integers(-8, 9, (P, D)) / 8.0).astype(np.float32)
    assert np.array_equal(SC.bf16_round(W32), W32)
    tn = rng.integers(0, 3, n)
    l0, s0, t0 = _plain_eval(Xb, tn, S.GINI, 3, 32)(W32)
    l1, s1, t1, g1 = SC.evaluate_screened(Xb, tn, S.GINI, 3, 32, k, z_bf16=False)(W32)
    assert np.array_equal(l0, l1) and np.array_equal(s0, s1) and np.array_equal(t0, t1)
    sel = SC.top_k(l0, k)
    assert np.array_equal(np.isfinite(g1), np.isin(np.arange(P), sel) & np.isfinite(l0))
    assert np.array_equal(g1[sel], l0[sel])


def test_screened_losses_track_float32_losses():
    """On Gaussian data the bfloat16 screen changes the best-threshold loss of
    a direction only a little, and the re-scored set holds the particles with
    the best float32 losses up to that noise."""
    rng = np.random.default_rng(11)
    X, y = inputs.cluster_mixture(3000, 16, 3, seed=3)
    Xb = SC.bf16_round(X)
    P, k = 128, 32
    W32 = inputs.random_unit_rows(P, 16, seed=12).astype(np.float32)
    l32, _, _ = _plain_eval(Xb, y, S.ENTROPY, 3, 64)(W32)
    Zs = S.project(Xb, SC.bf16_round(W32)).astype(np.float32)
    ls = np.array([S.scan_hist(Zs[:, p], y, 64, S.ENTROPY, 3)["loss"] for p in range(P)])
    assert np.max(np.abs(ls - l32)) < 0.05
    assert np.median(np.abs(ls - l32)) < 0.01
    best32 = set(np.argsort(l32)[:8].tolist())
    assert len(best32 & set(SC.top_k(ls, k).tolist())) >= 7
    del rng


def test_global_best_ignores_unrescored_particles():
    """A particle outside the re-scored set cannot become the global best even
    with the lowest loss; it still updates its personal best."""
    P, D = 6, 3
    x = np.eye(P, D) + 0.0
    loss = np.array([0.5, 0.1, 0.4, 0.3, 0.2, 0.6])
    gloss = np.array([0.5, np.inf, 0.4, np.inf, np.inf, np.inf])
    pb, pbl = x.copy() * 0, np.full(P, np.inf)
    gb, gbl, gp = np.zeros(D), np.array([np.inf]), np.array([-1])
    assert O.update_bests(x, loss, pb, pbl, gb, gbl, gp, gloss)
    assert gp[0] == 2 and gbl[0] == 0.4 and np.array_equal(gb, x[2])
    assert np.array_equal(pbl, loss) and np.array_equal(pb, x)


def test_screened_swarm_separates_planted_hyperplane():
    """End to end: with screening the swarm still finds a zero-loss direction
    for two classes split by a planted hyperplane."""
    rng = np.random.default_rng(13)
    n, D = 600, 6
    Xb = SC.bf16_round(rng.standard_normal((n, D)).astype(np.float32))
    a = np.array([1.0, -2.0, 0.5, 0.0, 1.5, -1.0])
    y = (Xb @ a > 0.05).astype(np.int64)
    ev = SC.evaluate_screened(Xb, y, S.GINI, 2, 0, 8)
    r = O.run_pso(ev, 32, D, 30, 0.7, 1.5, 1.5, seed=4, tree=0, node=0)
    assert r["loss"] == 0.0
    z = S.project(Xb, r["gbest"].astype(np.float32)[None, :])[:, 0].astype(np.float32)
    right = z >= r["thr"]
    assert len(np.unique(y[right])) == 1 and len(np.unique(y[~right])) == 1
