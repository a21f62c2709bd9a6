"""Oracle: particle swarm search over projection directions (Sec. III, Alg. 1).

Each particle's position is a candidate direction a (Sec. III-B); its loss is
the loss of the best threshold of the projected feature (oracle.split).

Readings of the paper used here (it leaves them open):
* synchronous swarm: all P particles are evaluated, then personal and global
  bests are updated, then all particles move with the same global best;
* Eq. (12) is read as x_{t+1} = x_t + v_{t+1} (the usual inertia-weight form;
  the printed v_t index is taken as a typo);
* r1, r2 are drawn per particle, per dimension and per move, uniform in [0, 1)
  with 24 bits, from Philox4x32-10 (oracle.philox);
* x is rescaled to unit norm after each move, since Eq. (2) asks for ||a|| = 1
  and the loss does not depend on the scale of a; v is left as is; a position
  of zero norm keeps its previous value;
* initial positions are N(0, I) draws (Box-Muller on Philox words) scaled to
  unit norm, initial velocities zero;
* strict "<" for personal and global bests; the lowest particle index wins a
  tie for the global best;
* T moves and T+1 evaluations.
"""
from __future__ import annotations

import numpy as np

from .philox import INIT_STREAM, philox4x32_10, pso_counter, seed_key, u24

TWO_PI = 6.283185307179586


def _words(seed, tree, node, t, P, D):
    """Philox words [P, ceil(D/2), 4] for every (particle, dimension pair)."""
    dh = (D + 1) // 2
    ctr = np.array([pso_counter(tree, node, t, p, 2 * m, D) for p in range(P) for m in range(dh)],
                   dtype=np.uint64).reshape(P, dh, 4)
    return philox4x32_10(ctr, seed_key(seed))


def uniforms(seed, tree, node, t, P, D):
    """r1, r2 [P, D] for the move numbered t (t = 1..T).

    Dimension pair m = d // 2 uses one Philox call: words (0, 1) give r1, r2 of
    dimension 2m and words (2, 3) give r1, r2 of dimension 2m + 1."""
    w = _words(seed, tree, node, t, P, D)
    r1 = np.empty((P, 2 * w.shape[1]))
    r2 = np.empty_like(r1)
    r1[:, 0::2], r2[:, 0::2] = u24(w[..., 0]), u24(w[..., 1])
    r1[:, 1::2], r2[:, 1::2] = u24(w[..., 2]), u24(w[..., 3])
    return r1[:, :D], r2[:, :D]


def normalize_rows(x):
    """x / ||x|| per row; the squared norm is summed in dimension order.
    Rows of zero norm are returned unchanged (flag False)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.zeros(x.shape[0])
    for d in range(x.shape[1]):
        s = s + x[:, d] * x[:, d]
    nrm = np.sqrt(s)
    ok = nrm > 0
    out = x.copy()
    out[ok] = x[ok] / nrm[ok, None]
    return out, ok


def init_positions(seed, tree, node, P, D, mask=None):
    """x0 [P, D]: Box-Muller normals from the INIT_STREAM words, unit rows.

    u1 = (w0 + 1/2) 2^-32, u2 = w1 2^-32; the pair is
    sqrt(-2 ln u1) * (cos(2 pi u2), sin(2 pi u2)) for dimensions 2m, 2m+1.
    mask [D] bool, if given: the normals of dimensions outside it are set to
    zero before the rows are scaled (a start in the span of the masked-in
    unit vectors, oracle.dft)."""
    w = _words(seed, tree, node, INIT_STREAM, P, D)
    u1 = (w[..., 0].astype(np.float64) + 0.5) * (2.0 ** -32)
    u2 = w[..., 1].astype(np.float64) * (2.0 ** -32)
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = TWO_PI * u2
    g = np.empty((P, 2 * w.shape[1]))
    g[:, 0::2] = rad * np.cos(ang)
    g[:, 1::2] = rad * np.sin(ang)
    g = g[:, :D]
    if mask is not None:
        g = np.where(np.asarray(mask, dtype=bool)[None, :], g, 0.0)
    x, _ = normalize_rows(g)
    return x


def update_bests(x, loss, pbest, pbest_loss, gbest, gbest_loss, gbest_p, gloss=None):
    """Personal bests (strict <) then the global best (argmin, lowest p on ties,
    taken only if strictly below the current global best).  One node; in place.
    gloss, if given, holds the losses eligible for the global best (a screened
    evaluation admits only its re-scored particles); by default it is loss.
    Returns True if the global best changed."""
    better = loss < pbest_loss
    pbest[better] = x[better]
    pbest_loss[better] = loss[better]
    g = loss if gloss is None else np.asarray(gloss, dtype=np.float64)
    p = int(np.argmin(g))
    if g[p] < gbest_loss[0]:
        gbest[:] = x[p]
        gbest_loss[0] = g[p]
        gbest_p[0] = p
        return True
    return False


def move(x, v, pbest, gbest, r1, r2, omega, c1, c2):
    """Eq. (11) then Eq. (12) and the unit-norm rescale; one node.

    v' = ((omega v) + ((c1 r1)(pB - x))) + ((c2 r2)(gB - x)), each operation
    rounded once in FP64, evaluated in that order."""
    a = omega * v
    b = (c1 * r1) * (pbest - x)
    c = (c2 * r2) * (gbest[None, :] - x)
    vn = (a + b) + c
    xn, ok = normalize_rows(x + vn)
    xn[~ok] = x[~ok]
    return xn, vn


def pso_step(x, v, pbest, pbest_loss, gbest, gbest_loss, gbest_p, loss, node_id,
             n_nodes, P, D, omega, c1, c2, seed, tree, it, do_move, gloss=None):
    """Batched step over n_nodes swarms laid out [n_nodes * P, D]; returns new
    arrays (inputs are not modified).  gloss [n_nodes * P]: optional losses
    eligible for the global best (see update_bests)."""
    x, v, pbest = x.copy(), v.copy(), pbest.copy()
    pbest_loss, gbest = pbest_loss.copy(), gbest.copy()
    gbest_loss, gbest_p = gbest_loss.copy(), gbest_p.copy()
    for j in range(n_nodes):
        s = slice(j * P, (j + 1) * P)
        xs, vs, pbs, pbl = x[s], v[s], pbest[s], pbest_loss[s]
        gb, gbl, gp = gbest[j], gbest_loss[j:j + 1], gbest_p[j:j + 1]
        update_bests(xs, loss[s], pbs, pbl, gb, gbl, gp, None if gloss is None else gloss[s])
        if do_move:
            r1, r2 = uniforms(seed, tree, int(node_id[j]), it, P, D)
            x[s], v[s] = move(xs, vs, pbs, gb, r1, r2, omega, c1, c2)
    return dict(x=x, v=v, pbest=pbest, pbest_loss=pbest_loss, gbest=gbest,
                gbest_loss=gbest_loss, gbest_p=gbest_p)


def run_pso(evaluate, P, D, T, omega, c1, c2, seed, tree, node, x0=None, target_loss=None):
    """Alg. 1 for one node.

    evaluate(W32 [P, D] float32) -> (loss [P], split [P], thr [P]) or
    (loss, split, thr, gloss) where gloss holds the losses eligible for the
    global best.  The directions handed to the evaluation are the float32
    images of the FP64 positions.  x0 replaces the random initial positions
    (rows are used as given).  With target_loss the loop stops after the
    first evaluation whose global-best loss is <= target_loss.
    Returns dict(gbest, loss, split, thr, p, evals, history)."""
    x = init_positions(seed, tree, node, P, D) if x0 is None else np.array(x0, dtype=np.float64)
    v = np.zeros_like(x)
    pbest = x.copy()
    pbest_loss = np.full(P, np.inf)
    gbest = x[0].copy()
    gbest_loss = np.array([np.inf])
    gbest_p = np.array([-1])
    g_split, g_thr = -1, np.float32(np.inf)
    history = []
    evals = 0
    for t in range(T + 1):
        out = evaluate(x.astype(np.float32))
        loss, split, thr = out[:3]
        gloss = out[3] if len(out) > 3 else None
        evals += 1
        loss = np.asarray(loss, dtype=np.float64)
        if update_bests(x, loss, pbest, pbest_loss, gbest, gbest_loss, gbest_p, gloss):
            g_split, g_thr = int(split[gbest_p[0]]), np.float32(thr[gbest_p[0]])
        history.append(float(gbest_loss[0]))
        if target_loss is not None and gbest_loss[0] <= target_loss:
            break
        if t < T:
            r1, r2 = uniforms(seed, tree, node, t + 1, P, D)
            x, v = move(x, v, pbest, gbest, r1, r2, omega, c1, c2)
    return dict(gbest=gbest, loss=float(gbest_loss[0]), split=g_split, thr=g_thr,
                p=int(gbest_p[0]), evals=evals, history=history)
