"""Pins of the APSO oracle (oracle.apso; CPU only).

* the directions of the c1 / c2 changes in each state are the paper's
  (Sec. III-B: exploration raises c1 and lowers c2, exploitation raises c1
  slightly and lowers c2, convergence raises both slightly, jumping-out lowers
  c1 and raises c2), with the bounds kept;
* mean distances against scipy's pairwise distances;
* the evolutionary factor's meaning: a global best at the centre of a cluster
  of particles reads convergence (f = 0), one far outside reads jumping-out;
* the inertia weight's closed-form end points and monotonicity; the
  memberships cover [0, 1] and each state holds its core interval;
* the elitist step moves one coordinate, keeps a unit norm, and its sigma
  falls linearly from 1 to 0.1;
* a run never loses its global best, T = 0 is the plain swarm's single
  evaluation, and on a smooth landscape the adaptive swarm converges.

Parity unpinned: the membership breakpoints, the hysteresis of `classify`, the
inertia law, the delta range and the sigma schedule are readings of the APSO
reference, which is not at hand.  `test_inertia_and_memberships` checks the
inertia end points against the oracle's own formula and the core intervals'
order only, so a shifted breakpoint or constant would still pass; what these
tests do pin is what the paper fixes and what holds mathematically.
"""
import math

import numpy as np
import pytest
from scipy.spatial.distance import pdist, squareform

from oracle import apso as A
from oracle import pso as O


@pytest.mark.parametrize("state", [1, 2, 3, 4])
def test_state_changes_follow_the_paper(state):
    d1, d2 = 0.08, 0.06
    c1, c2 = A.adapt(state, 2.0, 1.9, d1, d2)
    dc1, dc2 = c1 - 2.0, c2 - 1.9
    if state == A.EXPLORATION:
        assert dc1 > 0 and dc2 < 0
    elif state == A.EXPLOITATION:
        assert 0 < dc1 < d1 and dc2 < 0           # c1 up slightly
    elif state == A.CONVERGENCE:
        assert 0 < dc1 < d1 and 0 < dc2 < d2      # both up slightly
    else:
        assert dc1 < 0 and dc2 > 0
    # the clamp and the sum limit
    for s in (1, 2, 3, 4):
        for a, b in ((2.5, 2.5), (1.5, 1.5), (2.45, 1.52), (1.52, 2.45)):
            c1, c2 = A.adapt(s, a, b, 0.1, 0.1)
            assert 1.5 - 1e-12 <= c1 <= 2.5 and 1.5 - 1e-12 <= c2 <= 2.5
            assert c1 + c2 <= 4.0 + 1e-12


def test_mean_distances_against_scipy():
    rng = np.random.default_rng(0)
    for P, D in ((2, 3), (17, 5), (64, 33)):
        x = rng.standard_normal((P, D))
        ref = squareform(pdist(x)).sum(axis=1) / (P - 1)
        assert np.allclose(A.mean_distances(x), ref, rtol=1e-13, atol=0)


def test_evolutionary_factor_reads_the_swarm():
    rng = np.random.default_rng(1)
    cloud = rng.standard_normal((30, 4)) * 0.1
    centre = np.zeros((1, 4))
    far = np.full((1, 4), 5.0)
    x = np.vstack([centre, cloud])            # best at the centre of the cluster
    f = A.evolutionary_factor(A.mean_distances(x), 0)
    assert f == 0.0 and A.classify(f, A.EXPLORATION) == A.CONVERGENCE
    x = np.vstack([far, cloud])               # best far from the cluster
    f = A.evolutionary_factor(A.mean_distances(x), 0)
    assert f == 1.0 and A.classify(f, A.CONVERGENCE) == A.JUMPING_OUT
    # all particles equally spread: no information, f = 0
    sq = np.array([[1.0, 0], [0, 1.0], [-1.0, 0], [0, -1.0]])
    assert A.evolutionary_factor(A.mean_distances(sq), 2) == 0.0


def test_inertia_and_memberships():
    assert A.inertia(0.0) == pytest.approx(0.4, rel=1e-15)
    assert A.inertia(1.0) == pytest.approx(1.0 / (1.0 + 1.5 * math.exp(-2.6)), rel=1e-15)
    fs = np.linspace(0, 1, 1001)
    w = [A.inertia(f) for f in fs]
    assert all(b > a for a, b in zip(w, w[1:]))
    for f in fs:
        mu = A.memberships(f)
        assert all(0.0 <= m <= 1.0 for m in mu) and max(mu) > 0, f
    # core intervals: each state alone with membership one
    for f, s in ((0.05, A.CONVERGENCE), (0.35, A.EXPLOITATION), (0.65, A.EXPLORATION),
                 (0.95, A.JUMPING_OUT)):
        mu = A.memberships(f)
        assert mu[s - 1] == 1.0 and sum(mu) == 1.0
        for prev in (1, 2, 3, 4):
            assert A.classify(f, prev) == s
    # an overlap keeps the previous state while it still applies
    assert A.classify(0.5, A.EXPLOITATION) == A.EXPLOITATION
    assert A.classify(0.5, A.EXPLORATION) == A.EXPLORATION
    assert A.classify(0.75, A.EXPLORATION) == A.EXPLORATION
    assert A.classify(0.75, A.CONVERGENCE) == A.EXPLORATION     # larger membership


def test_elite_step():
    g = O.normalize_rows(np.arange(1.0, 7.0)[None, :])[0][0]
    e = A.elite(g, 2, 0.7, 0.5)
    assert np.linalg.norm(e) == pytest.approx(1.0, rel=1e-15)
    raw = g.copy()
    raw[2] += 2.0 * 0.5 * 0.7
    assert np.allclose(e, raw / np.linalg.norm(raw), rtol=0, atol=1e-15)
    assert A.sigma(0, 10) == 1.0 and A.sigma(10, 10) == pytest.approx(0.1, rel=1e-15)
    assert A.sigma(5, 10) == pytest.approx(0.55, rel=1e-15)
    # the draws: deltas in [0.05, 0.1], dimension in range, normals ~ N(0, 1)
    gs = []
    for t in range(1, 400):
        d1, d2, dim, gv = A.draws(3, 1, 7, t, 13)
        assert 0.05 <= d1 < 0.1 and 0.05 <= d2 < 0.1 and 0 <= dim < 13
        gs.append(gv)
    assert abs(np.mean(gs)) < 0.2 and abs(np.std(gs) - 1) < 0.15


def _angle_loss(target):
    target = target / np.linalg.norm(target)

    def ev(W32):
        W = W32.astype(np.float64)
        cos = (W @ target) / np.linalg.norm(W, axis=1)
        loss = 1.0 - cos
        return loss, np.zeros(len(W), dtype=np.int64), np.zeros(len(W), dtype=np.float32)
    return ev


def test_run_keeps_its_best_and_converges():
    rng = np.random.default_rng(2)
    target = rng.standard_normal(6)
    log = []
    r = A.run_apso(_angle_loss(target), 24, 6, 40, seed=5, tree=0, node=3, log=log)
    h = r["history"]
    assert all(b <= a for a, b in zip(h, h[1:]))
    assert r["loss"] < 1e-3
    assert set(r["states"]) <= {1, 2, 3, 4} and len(r["states"]) == 40
    # the states follow the swarm's spread: convergence appears once it gathers
    assert A.CONVERGENCE in r["states"]
    for a in log:
        assert 1.5 - 1e-12 <= a["c1"] <= 2.5 and 1.5 - 1e-12 <= a["c2"] <= 2.5
        assert 0.4 <= a["omega"] < 0.9
        assert (a["elite"] is not None) == (a["state"] == A.CONVERGENCE)
    # T = 0: the start and one evaluation, exactly the plain swarm's
    p0 = O.run_pso(_angle_loss(target), 24, 6, 0, 0.7, 1.5, 1.5, 5, 0, 3)
    a0 = A.run_apso(_angle_loss(target), 24, 6, 0, 5, 0, 3)
    assert np.array_equal(p0["gbest"], a0["gbest"]) and p0["loss"] == a0["loss"]


def test_apso_tree_root_is_the_apso_run():
    from oracle import split as S
    from oracle import tree as T
    from paper_2208_07023_amd import inputs
    X, y, _ = inputs.two_class_gaussian(400, 5, seed=4)
    prm = T.TreeParams(crit=S.GINI, K=2, max_depth=2, min_node=8, P=12, T=6, bins=32, seed=9,
                       search=1)
    tr = T.grow_tree(X, y, prm).arrays()
    r = A.run_apso(T.evaluate_node(X, y, prm), 12, 5, 6, 9, 0, 0)
    assert np.array_equal(tr["w"][0], r["gbest"].astype(np.float32))
    assert tr["split_loss"][0] == r["loss"] < tr["impurity"][0]
    assert tr["n"][1] + tr["n"][2] == 400


def test_run_in_a_subspace_stays_there():
    from oracle import dft as OD
    rng = np.random.default_rng(6)
    D, dims = 9, np.array([7, 2, 4])
    target = np.zeros(D)
    target[dims] = rng.standard_normal(3)
    x0 = OD.subspace_start(3, 0, 1, 16, D, dims)
    log = []
    r = A.run_apso(_angle_loss(target), 16, D, 30, 3, 0, 1, x0=x0, log=log, dims=dims)
    out = np.setdiff1d(np.arange(D), dims)
    assert np.all(r["gbest"][out] == 0.0)
    assert any(a["elite"] is not None for a in log)
    for a in log:
        if a["elite"] is not None:
            assert np.all(a["elite"][out] == 0.0)
    assert r["loss"] < 1e-3
