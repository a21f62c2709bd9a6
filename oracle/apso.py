"""Oracle: adaptive particle swarm optimisation (APSO) of one node (Sec. III-B).

The paper adopts APSO as an alternative swarm: before each iteration the
distribution of the particles is classified as one of four evolutionary
states (exploration, exploitation, convergence, jumping-out) and c1, c2 change
with the state: exploration raises c1 and lowers c2; exploitation raises c1
slightly and lowers c2; convergence raises both slightly and applies an
elitist learning step to the global best; jumping-out lowers c1 and raises
c2.  The state estimation, the sizes of the changes, the inertia weight and
the elitist step are left to the APSO reference (Zhan, Zhang, Li and Chung,
"Adaptive Particle Swarm Optimization", IEEE Trans. SMC-B, 2009).  Readings of
this build, from that method as published:

* evolutionary state estimation: d_i = mean Euclidean distance of particle i
  to the other P-1 particles; f = (d_g - d_min) / (d_max - d_min) with g the
  particle that holds the global best (f = 0 when d_max = d_min);
* fuzzy memberships of f (piecewise linear, see `memberships`); the state is
  the previous one while its membership stays positive, else the state of
  largest membership (the lower state number on ties); the first state is
  exploration;
* inertia omega = 1 / (1 + 1.5 exp(-2.6 f)); c1 and c2 start at 2 and change
  by delta1, delta2 ~ U[0.05, 0.1] ("slightly": half of that), are clamped to
  [1.5, 2.5] and scaled to sum 4 when their sum exceeds 4;
* elitist learning (convergence only): one coordinate d (uniform) of the
  global best is moved by (x_max - x_min) sigma N(0, 1), with x in [-1, 1]
  (range 2) and sigma falling linearly from 1 to 0.1 over the run
  (sigma = 1 - 0.9 t / T at move t = 1..T), then scaled to unit norm; the
  candidate replaces the particle with the highest loss of the evaluation
  (lowest index on ties) after the move, with zero velocity, and is
  evaluated with the swarm at the next iteration;
* the move itself is Eqs. (11)-(12) with the state's omega, c1, c2 and the
  same r1, r2 draws as the plain swarm (oracle.pso);
* the extra draws of move t come from Philox4x32-10 counters
  (0, APSO_STREAM + t, node, tree): delta1 = 0.05 + 0.05 u24(w0),
  delta2 = 0.05 + 0.05 u24(w1), d = floor(w2 D / 2^32) (with the swarm in
  the span of a node's top n DFT channels, Alg. 2: the floor(w2 n / 2^32)-th
  of those channels, so the step stays in the subspace); and
  (1, APSO_STREAM + t, node, tree): the normal draw from words 0 and 1 as in
  the swarm's start (Box-Muller, cosine branch).

Parity unpinned: the membership breakpoints of `memberships`, the hysteresis
rule of `classify`, the inertia law of `inertia`, the delta range of the c1/c2
changes, the clamp and sum limits, and the elitist step's sigma schedule are
readings of the APSO reference, which is not at hand, recalled rather than
checked against it.  The tests pin only what the paper itself fixes (the four
states and the directions in which c1 and c2 move in each) and what holds
mathematically (distances, the evolutionary factor's range and extremes, the
unit norm of the elitist candidate); a shifted breakpoint or inertia constant
would pass them.  The GPU follows these readings and is compared with them.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import philox4x32_10, seed_key, u24
from .pso import init_positions, move, normalize_rows, uniforms, update_bests

EXPLORATION, EXPLOITATION, CONVERGENCE, JUMPING_OUT = 1, 2, 3, 4
APSO_STREAM = 0x20000000
C_MIN, C_MAX, C_SUM = 1.5, 2.5, 4.0
SIGMA_MAX, SIGMA_MIN = 1.0, 0.1
X_RANGE = 2.0
TWO_PI = 6.283185307179586


def mean_distances(x):
    """d_i = (1 / (P - 1)) sum_{j != i} ||x_i - x_j|| (P >= 2)."""
    x = np.asarray(x, dtype=np.float64)
    P = x.shape[0]
    diff = x[:, None, :] - x[None, :, :]
    dist = np.sqrt(np.sum(diff * diff, axis=2))
    return dist.sum(axis=1) / (P - 1)


def evolutionary_factor(d, g: int):
    dmin, dmax = float(np.min(d)), float(np.max(d))
    if not dmax > dmin:
        return 0.0
    return (float(d[g]) - dmin) / (dmax - dmin)


def memberships(f: float):
    """(mu_exploration, mu_exploitation, mu_convergence, mu_jumping_out)."""
    if f <= 0.4:
        m1 = 0.0
    elif f <= 0.6:
        m1 = 5.0 * f - 2.0
    elif f <= 0.7:
        m1 = 1.0
    elif f <= 0.8:
        m1 = -10.0 * f + 8.0
    else:
        m1 = 0.0
    if f <= 0.2:
        m2 = 0.0
    elif f <= 0.3:
        m2 = 10.0 * f - 2.0
    elif f <= 0.4:
        m2 = 1.0
    elif f <= 0.6:
        m2 = -5.0 * f + 3.0
    else:
        m2 = 0.0
    if f <= 0.1:
        m3 = 1.0
    elif f <= 0.3:
        m3 = -5.0 * f + 1.5
    else:
        m3 = 0.0
    if f <= 0.7:
        m4 = 0.0
    elif f <= 0.9:
        m4 = 5.0 * f - 3.5
    else:
        m4 = 1.0
    return (m1, m2, m3, m4)


def classify(f: float, prev: int) -> int:
    mu = memberships(f)
    if mu[prev - 1] > 0.0:
        return prev
    best = 1
    for s in (2, 3, 4):
        if mu[s - 1] > mu[best - 1]:
            best = s
    return best


def inertia(f: float) -> float:
    return 1.0 / (1.0 + 1.5 * math.exp(-2.6 * f))


def adapt(state: int, c1: float, c2: float, d1: float, d2: float):
    """c1, c2 after one state's change, clamp and sum limit."""
    if state == EXPLORATION:
        c1, c2 = c1 + d1, c2 - d2
    elif state == EXPLOITATION:
        c1, c2 = c1 + 0.5 * d1, c2 - 0.5 * d2
    elif state == CONVERGENCE:
        c1, c2 = c1 + 0.5 * d1, c2 + 0.5 * d2
    else:
        c1, c2 = c1 - d1, c2 + d2
    c1 = min(max(c1, C_MIN), C_MAX)
    c2 = min(max(c2, C_MIN), C_MAX)
    if c1 + c2 > C_SUM:
        s = C_SUM / (c1 + c2)
        c1, c2 = c1 * s, c2 * s
    return c1, c2


def draws(seed: int, tree: int, node: int, t: int, D: int, dims=None):
    """(delta1, delta2, elite dimension, normal draw) of move t; with dims
    (the swarm's coordinates, e.g. a node's top DFT channels) the dimension is
    dims[floor(w2 len(dims) / 2^32)]."""
    ctr = np.array([[0, APSO_STREAM + t, node, tree], [1, APSO_STREAM + t, node, tree]],
                   dtype=np.uint64)
    w = philox4x32_10(ctr, seed_key(seed))
    d1 = 0.05 + 0.05 * float(u24(w[0, 0]))
    d2 = 0.05 + 0.05 * float(u24(w[0, 1]))
    if dims is None:
        dim = int((int(w[0, 2]) * D) >> 32)
    else:
        dim = int(dims[(int(w[0, 2]) * len(dims)) >> 32])
    u1 = (float(w[1, 0]) + 0.5) * (2.0 ** -32)
    u2 = float(w[1, 1]) * (2.0 ** -32)
    g = math.sqrt(-2.0 * math.log(u1)) * math.cos(TWO_PI * u2)
    return d1, d2, dim, g


def sigma(t: int, T: int) -> float:
    return SIGMA_MAX - (SIGMA_MAX - SIGMA_MIN) * (t / T)


def elite(gbest, dim: int, g: float, sig: float):
    e = np.array(gbest, dtype=np.float64)
    e[dim] = e[dim] + (X_RANGE * sig) * g
    out, ok = normalize_rows(e[None, :])
    return out[0] if ok[0] else np.array(gbest, dtype=np.float64)


def worst_particle(loss) -> int:
    loss = np.asarray(loss, dtype=np.float64)
    return int(np.argmax(np.where(np.isnan(loss), np.inf, loss)))


def apso_adapt(x, gbest, gbest_p: int, loss, state: int, c1: float, c2: float,
               seed: int, tree: int, node: int, t: int, T: int, dims=None):
    """One state estimation and parameter change before move t (1..T); dims:
    the coordinates the swarm lives in (None: all).
    Returns dict(d, f, state, omega, c1, c2, worst, elite or None)."""
    d = mean_distances(x)
    f = evolutionary_factor(d, max(0, int(gbest_p)))
    st = classify(f, state)
    d1, d2, dim, g = draws(seed, tree, node, t, x.shape[1], dims)
    c1n, c2n = adapt(st, c1, c2, d1, d2)
    out = dict(d=d, f=f, state=st, omega=inertia(f), c1=c1n, c2=c2n, worst=worst_particle(loss),
               elite=None)
    if st == CONVERGENCE:
        out["elite"] = elite(gbest, dim, g, sigma(t, T))
    return out


def run_apso(evaluate, P, D, T, seed, tree, node, x0=None, log=None, dims=None):
    """APSO for one node; evaluate as in oracle.pso.run_pso.  dims: the
    coordinates the swarm lives in (a start in their span, x0, keeps the others
    at zero; the elitist step perturbs one of them).
    Returns dict(gbest, loss, split, thr, p, evals, history, states)."""
    x = init_positions(seed, tree, node, P, D) if x0 is None else np.array(x0, dtype=np.float64)
    v = np.zeros_like(x)
    pbest = x.copy()
    pbest_loss = np.full(P, np.inf)
    gbest = x[0].copy()
    gbest_loss = np.array([np.inf])
    gbest_p = np.array([-1])
    g_split, g_thr = -1, np.float32(np.inf)
    state, c1, c2 = EXPLORATION, 2.0, 2.0
    history, states = [], []
    for t in range(T + 1):
        loss, split, thr = evaluate(x.astype(np.float32))[:3]
        loss = np.asarray(loss, dtype=np.float64)
        if update_bests(x, loss, pbest, pbest_loss, gbest, gbest_loss, gbest_p):
            g_split, g_thr = int(split[gbest_p[0]]), np.float32(thr[gbest_p[0]])
        history.append(float(gbest_loss[0]))
        if t == T:
            break
        a = apso_adapt(x, gbest, gbest_p[0], loss, state, c1, c2, seed, tree, node, t + 1, T,
                       dims)
        if log is not None:
            log.append(a)
        state, c1, c2 = a["state"], a["c1"], a["c2"]
        states.append(state)
        r1, r2 = uniforms(seed, tree, node, t + 1, P, D)
        x, v = move(x, v, pbest, gbest, r1, r2, a["omega"], c1, c2)
        if a["elite"] is not None:
            x[a["worst"]] = a["elite"]
            v[a["worst"]] = 0.0
    return dict(gbest=gbest, loss=float(gbest_loss[0]), split=g_split, thr=g_thr,
                p=int(gbest_p[0]), evals=T + 1, history=history, states=states)
