"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This module holds input recipes only: random draws with numpy's PCG64
(`numpy.random.default_rng(seed)`), shaping and storage-format rounding.  It
contains none of the method's arithmetic (no projection, binning, impurity or
swarm update), so both sides of every parity check can take their inputs from
here without sharing any computation.

The paper measures on small public tabular sets (Sec. V) that are not used
here; these generators are scaled-up stand-ins with the structure the workloads
name (Gaussian class mixtures, an absolute-projection regression target and a
low-rank-covariance many-class mixture).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


# --------------------------------------------------------------------------
# storage formats
# --------------------------------------------------------------------------
def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even).

    Returns the 16-bit patterns as uint16.  NaNs are not produced by any
    generator here, so no NaN special case is needed.
    """
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    # finite inputs: u + 0x8000 cannot wrap below 0xFFFF8000 (a NaN pattern)
    r = u + (np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1)))
    return (r >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Exact widening of bfloat16 bit patterns to float32."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


# --------------------------------------------------------------------------
# classification mixtures
# --------------------------------------------------------------------------
def balanced_labels(n: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """Exactly balanced labels (counts differ by at most one), randomly ordered."""
    y = (np.arange(n) % k).astype(np.int32)
    rng.shuffle(y)
    return y


def two_class_gaussian(n: int = 1000, d: int = 8, seed: int = 0):
    """Two classes, class means ~N(0, I), unit isotropic covariance, balanced.

    Returns (X float32 [n,d], y int32 [n], means float64 [2,d]).
    """
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((2, d))
    y = balanced_labels(n, 2, rng)
    X = means[y] + rng.standard_normal((n, d))
    return X.astype(np.float32), y, means


def cluster_mixture(n: int, d: int, k: int, clusters_per_class: int = 4,
                    mean_std: float = 2.0, var_lo: float = 0.5, var_hi: float = 2.0,
                    seed: int = 0):
    """K classes, each a mixture of equally weighted Gaussian clusters.

    Cluster means ~N(0, mean_std^2 I); diagonal covariances with per-dimension
    variances ~U[var_lo, var_hi].  Labels balanced.  Returns (X f32, y i32).
    """
    rng = np.random.default_rng(seed)
    c = clusters_per_class
    means = rng.standard_normal((k, c, d)) * mean_std
    variances = rng.uniform(var_lo, var_hi, size=(k, c, d))
    y = balanced_labels(n, k, rng)
    cl = rng.integers(0, c, size=n)
    X = means[y, cl] + rng.standard_normal((n, d)) * np.sqrt(variances[y, cl])
    return X.astype(np.float32), y


def lowrank_mixture(n: int, d: int = 256, k: int = 10, rank: int = 16, seed: int = 0,
                    chunk: int = 1 << 18):
    """K classes with means ~N(0, I) and a shared covariance L L^T + diag(delta).

    L [d, rank] has entries ~N(0, 1/rank); delta ~U[0.5, 2].  Generated in
    chunks so multi-million-row sets stay within a few GB of host memory.
    Returns (X bf16 bits uint16 [n,d], y int32 [n]).
    """
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((k, d)).astype(np.float32)
    L = (rng.standard_normal((d, rank)) / np.sqrt(rank)).astype(np.float32)
    delta = rng.uniform(0.5, 2.0, size=d).astype(np.float32)
    y = balanced_labels(n, k, rng)
    out = np.empty((n, d), dtype=np.uint16)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        g = rng.standard_normal((e - s, rank), dtype=np.float32)
        h = rng.standard_normal((e - s, d), dtype=np.float32)
        x = means[y[s:e]] + g @ L.T + h * np.sqrt(delta)
        out[s:e] = f32_to_bf16_bits(x)
    return out, y


# --------------------------------------------------------------------------
# regression
# --------------------------------------------------------------------------
def abs_direction_regression(n: int, d: int = 128, n_dirs: int = 8, noise: float = 0.1,
                             seed: int = 0, chunk: int = 1 << 18):
    """x ~N(0, I); y = sum_k |x . u_k| + N(0, noise^2), u_k random unit vectors.

    X is stored float32 and y float64; y is computed from the float32 X.
    Returns (X f32 [n,d], y f64 [n]).
    """
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n_dirs, d))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    X = np.empty((n, d), dtype=np.float32)
    y = np.empty(n, dtype=np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        x = rng.standard_normal((e - s, d)).astype(np.float32)
        X[s:e] = x
        y[s:e] = np.abs(x.astype(np.float64) @ U.T).sum(axis=1) + noise * rng.standard_normal(e - s)
    return X, y


def friedman1(n: int, d: int = 10, noise: float = 1.0, seed: int = 0):
    """Friedman's first regression function (Friedman, Ann. Statist. 1991):
    x ~U[0, 1]^d (d >= 5, only the first five inputs matter),
    y = 10 sin(pi x1 x2) + 20 (x3 - 1/2)^2 + 10 x4 + 5 x5 + N(0, noise^2).
    y is computed from the float32 X.  Returns (X f32 [n,d], y f64 [n])."""
    if d < 5:
        raise ValueError("friedman1 needs d >= 5")
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(n, d)).astype(np.float32)
    x = X.astype(np.float64)
    y = (10.0 * np.sin(np.pi * x[:, 0] * x[:, 1]) + 20.0 * (x[:, 2] - 0.5) ** 2
         + 10.0 * x[:, 3] + 5.0 * x[:, 4] + noise * rng.standard_normal(n))
    return X, y


# --------------------------------------------------------------------------
# small fixtures for parity tests
# --------------------------------------------------------------------------
def random_unit_rows(p: int, d: int, seed: int) -> np.ndarray:
    """Rows ~N(0, I) scaled to unit norm (float64)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((p, d))
    return w / np.linalg.norm(w, axis=1, keepdims=True)


def integer_matrix(rows: int, cols: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Integers uniform in [lo, hi] stored as float32 (exact)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(rows, cols)).astype(np.float32)


def segment_offsets(sizes) -> np.ndarray:
    """CSR row offsets [n_nodes+1] (int64) for consecutive node sizes."""
    return np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64))]).astype(np.int64)


def ragged_sizes(n_nodes: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=n_nodes).astype(np.int64)


def projected_features(n: int, p: int, seed: int, kind: str = "gauss") -> np.ndarray:
    """Synthetic projected-feature matrices Z [n, p] (float32).

    kind: "gauss" (continuous), "dups" (heavy duplication: values on a coarse
    grid), "const" (every column constant), "ints" (integers 0..255).
    """
    rng = np.random.default_rng(seed)
    if kind == "gauss":
        return (rng.standard_normal((n, p)) * rng.uniform(0.1, 10.0, size=p)
                + rng.uniform(-5, 5, size=p)).astype(np.float32)
    if kind == "dups":
        return (rng.integers(-6, 7, size=(n, p)) * 0.25).astype(np.float32)
    if kind == "const":
        return np.broadcast_to(rng.standard_normal(p).astype(np.float32), (n, p)).copy()
    if kind == "ints":
        return rng.integers(0, 256, size=(n, p)).astype(np.float32)
    raise ValueError(kind)


@dataclass
class PsoState:
    x: np.ndarray          # [nn*P, D] f64 positions (unit rows)
    v: np.ndarray          # [nn*P, D] f64 velocities
    pbest: np.ndarray      # [nn*P, D]
    pbest_loss: np.ndarray # [nn*P]
    gbest: np.ndarray      # [nn, D]
    gbest_loss: np.ndarray # [nn]
    gbest_p: np.ndarray    # [nn] int32
    loss: np.ndarray       # [nn*P] current losses


def random_pso_state(n_nodes: int, p: int, d: int, seed: int, ties: bool = False) -> PsoState:
    """A random mid-run swarm state.  With ties=True many losses coincide."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n_nodes * p, d))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    v = 0.3 * rng.standard_normal((n_nodes * p, d))
    pb = rng.standard_normal((n_nodes * p, d))
    pb /= np.linalg.norm(pb, axis=1, keepdims=True)
    if ties:
        loss = rng.integers(0, 4, size=n_nodes * p) / 8.0
        pbl = rng.integers(0, 4, size=n_nodes * p) / 8.0
    else:
        loss = rng.uniform(0, 1, size=n_nodes * p)
        pbl = rng.uniform(0, 1, size=n_nodes * p)
    gb = rng.standard_normal((n_nodes, d))
    gb /= np.linalg.norm(gb, axis=1, keepdims=True)
    gbl = np.minimum(pbl.reshape(n_nodes, p).min(axis=1), rng.uniform(0, 1, size=n_nodes))
    return PsoState(x, v, pb, pbl, gb, gbl, np.zeros(n_nodes, dtype=np.int32), loss)
