"""Python binding of libslm.so (C ABI in include/slm.h).

Argument marshalling only: every step of the split search runs in the HIP
kernels of the library.  Tensors are torch device tensors (torch provides the
device memory and the current HIP stream).  If the library is missing or no
GPU is visible the calls raise; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslm.so")

F32, BF16, F64, I32 = 0, 1, 2, 3
GINI, ENTROPY, MSE = 0, 1, 2
Z_ROWS, Z_TILED, Z_TILED8, Z_TILED8_BF16 = 0, 1, 2, 3
TIMING_SLOTS = 12   # slm_tree_out.timing entries (SLM_TIMING_SLOTS)
STATUS = {0: "SLM_OK", 1: "SLM_E_INVALID", 2: "SLM_E_SHAPE", 3: "SLM_E_DTYPE",
          4: "SLM_E_NOMEM", 5: "SLM_E_HIP", 6: "SLM_E_UNSUPPORTED"}


class SlmError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class TreeParams(ctypes.Structure):
    _fields_ = [("crit", ctypes.c_int32), ("K", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("min_node", ctypes.c_int32), ("P", ctypes.c_int32), ("T", ctypes.c_int32),
                ("bins", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rescore_k", ctypes.c_int32), ("omega", ctypes.c_double),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("tree", ctypes.c_uint32), ("use_graph", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("proposal", ctypes.c_int32),
                ("n_seeds", ctypes.c_int32), ("mlp_hidden", ctypes.c_int32),
                ("mlp", ctypes.c_void_p), ("dft_top_n", ctypes.c_int32),
                ("ps_pd", ctypes.c_void_p), ("ps_amax", ctypes.c_void_p), ("ps_R", ctypes.c_int32),
                ("apso", ctypes.c_int32)]


class TreeOut(ctypes.Structure):
    _fields_ = [("max_nodes", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("w", ctypes.c_void_p), ("thr", ctypes.c_void_p), ("left", ctypes.c_void_p),
                ("right", ctypes.c_void_p), ("leaf", ctypes.c_void_p), ("n", ctypes.c_void_p),
                ("impurity", ctypes.c_void_p), ("split_loss", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("heap", ctypes.c_void_p),
                ("timing", ctypes.c_void_p), ("sample_splits", ctypes.c_void_p),
                ("stats", ctypes.c_void_p), ("sigma", ctypes.c_void_p)]


_lib = None
_VP, _I32, _I64, _U32, _U64, _D, _SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                        ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                        ctypes.c_size_t)

_SIGS = {
    "slm_version": ([], ctypes.c_char_p),
    "slm_last_error": ([], ctypes.c_char_p),
    "slm_project": ([_VP, _I32, _I64, _I32, _VP, _I32, _VP, _I32, _I32, _VP, _I32, _VP, _VP, _VP],
                    _I32),
    "slm_split_scan_workspace": ([_I64, _I32, _I32, _I32, _I32, _I32], _SZ),
    "slm_split_scan": ([_VP, _I32, _VP, _VP, _VP, _I32, _I32, _I64, _VP, _I32, _I32, _I32, _I32,
                        _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP], _I32),
    "slm_pso_init": ([_VP] * 7 + [_VP, _I32, _I32, _I32, _U64, _U32, _VP, _I32, _VP], _I32),
    "slm_pso_init_subspace": ([_VP] * 7 + [_VP, _I32, _I32, _I32, _U64, _U32, _VP, _I32, _VP,
                                           _I32, _VP], _I32),
    "slm_dft_select_workspace": ([_I64, _I32, _I32, _I32, _I32, _I32], _SZ),
    "slm_ps_tables": ([_I32, _D, _VP, _VP, _VP], _I32),
    "slm_autotune_set": ([_I32, ctypes.c_char_p], _I32),
    "slm_autotune_plans": ([], _I32),
    "slm_split_scan_noalloc_max_bytes": ([], _SZ),
    "slm_split_scan_noalloc": ([_VP, _I32, _VP, _VP, _VP, _I32, _I32, _I64, _VP, _I32, _I32, _I32,
                                _I32, _VP, _VP, _VP, _VP, _VP, _VP], _I32),
    "slm_boost_scores": ([_VP, _VP, _VP, _VP, _VP, _I32, _VP, _I32, _I32, _I32, _VP, _D, _VP, _I64,
                          _VP, _VP, _VP], _I32),
    "slm_ps_candidates": ([_VP, _VP, _I32, _VP, _I32, _I32, _I32, _VP, _I32, _VP, _VP, _U64, _U32,
                           _U32, _VP], _I32),
    "slm_dft_select": ([_VP, _I64, _I32, _VP, _I32, _VP, _I32, _I32, _I32, _I32, _I32, _VP, _VP,
                        _VP, _SZ, _VP], _I32),
    "slm_pso_step": ([_VP] * 7 + [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _I32, _I32, _I32, _D, _D,
                                  _D, _U64, _U32, _U32, _I32, _VP, _I32, _VP], _I32),
    "slm_apso_workspace": ([_I32, _I32], _SZ),
    "slm_apso_step": ([_VP] * 8 + [_VP, _I32, _I32, _I32, _U64, _U32, _U32, _U32, _VP, _VP, _VP,
                                   _VP, _VP, _VP, _VP, _I32, _VP, _SZ, _VP, _I32, _VP], _I32),
    "slm_screen_select": ([_VP, _I32, _I32, _I32, _VP, _VP], _I32),
    "slm_screen_gather": ([_VP, _VP, _I32, _I32, _I32, _I32, _VP, _VP], _I32),
    "slm_screen_merge": ([_VP, _VP, _VP, _VP, _I32, _I32, _I32, _VP, _VP, _VP, _VP, _VP], _I32),
    "slm_grow_tree_workspace": ([ctypes.POINTER(TreeParams), _I64, _I32], _SZ),
    "slm_grow_tree": ([_VP, _I32, _I64, _I32, _VP, _I32, ctypes.POINTER(TreeParams), _VP, _SZ,
                       ctypes.POINTER(TreeOut), _VP], _I32),
    "slm_predict": ([_VP, _VP, _VP, _VP, _I32, _I32, _VP, _I64, _VP, _VP], _I32),
    "slm_grow_forest_workspace": ([ctypes.POINTER(TreeParams), _I64, _I32, _I32], _SZ),
    "slm_grow_forest": ([_VP, _I32, _I64, _I32, _VP, _I32, ctypes.POINTER(TreeParams), _I32, _I32,
                         _VP, _SZ, _VP, ctypes.POINTER(TreeOut), _VP, _VP], _I32),
    "slm_forest_predict": ([_VP, _VP, _VP, _VP, _VP, _I32, _VP, _I32, _I32, _I32, _VP, _I64, _VP,
                            _VP, _VP], _I32),
    "slm_boost_workspace": ([ctypes.POINTER(TreeParams), _I64, _I32, _I32], _SZ),
    "slm_boost": ([_VP, _I64, _I32, _VP, _I32, _I32, ctypes.POINTER(TreeParams), _I32, _D, _VP,
                   _SZ, _VP, _VP, ctypes.POINTER(TreeOut), _VP, _VP], _I32),
    "slm_evaluate": ([_VP, _I64, _I32, _VP, _VP, _I32, _I32, _VP, _I32, _I32, _I32, _VP, _VP, _VP,
                      _VP, _VP, _VP, _SZ, _VP], _I32),
    "slm_search_nodes_workspace": ([ctypes.POINTER(TreeParams), _I64, _I32, _I32], _SZ),
    "slm_search_nodes": ([_VP, _I32, _I64, _I32, _VP, _I32, _VP, _VP, _I32,
                          ctypes.POINTER(TreeParams), _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP],
                         _I32),
    "slm_node_stats_workspace": ([_I32, _I32, _I32], _SZ),
    "slm_node_stats": ([_VP, _I32, _I64, _I32, _VP, _I32, _VP, _I32, _VP, _VP, _VP, _SZ, _VP], _I32),
    "slm_mlp_param_count": ([_I32, _I32, _I32], _I64),
    "slm_mlp_forward": ([_VP, _I32, _I32, _I32, _VP, _I32, _I32, _VP, _VP, _VP], _I32),
    "slm_mlp_backward": ([_VP, _I32, _I32, _I32, _VP, _I32, _VP, _VP, _VP, _VP, _VP], _I32),
    "slm_wta_loss": ([_VP, _VP, _I32, _I32, _I32, ctypes.c_float, ctypes.c_float, _VP, _VP, _VP],
                     _I32),
    "slm_proposal_targets": ([_VP, _VP, _I32, _I32, _VP, _VP], _I32),
    "slm_adam_step": ([_VP, _VP, _VP, _VP, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                       ctypes.c_float, _I32, _VP], _I32),
    "slm_proposal_seeds": ([_VP, _VP, _I32, _I32, _I32, _I32, _VP, _VP, _VP, _I32, _VP], _I32),
}


def load(path: str = LIB_PATH):
    """Load libslm.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        for name, (args, res) in _SIGS.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def _check(st: int, where: str):
    if st != 0:
        raise SlmError(st, where, _lib.slm_last_error().decode())


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _xdtype(X):
    if X.dtype == torch.float32:
        return F32
    if X.dtype == torch.bfloat16:
        return BF16
    raise TypeError("X must be float32 or bfloat16")


# ------------------------------------------------------------------ project
def _tile_width(tiled):
    """(tile width, bfloat16): 0 (row-major), 32 (tiled=True or 32), 8, or
    "bf16" (8-wide tiles of bfloat16)."""
    if tiled == "bf16":
        return 8, True
    w = 32 if tiled is True else int(tiled or 0)
    if w not in (0, 8, 32):
        raise ValueError("tiled must be False, True (32), 32, 8 or 'bf16'")
    return w, False


def project(X, W, row_off, P: int, tiled=False):
    """Z = per-node X W^T, zmin/zmax [n_nodes*P] (Eq. (1)).  Z is [N, P], or
    with tiled=True (or 32) the particle-tiled [ceil(P/32), N, 32]
    (SLM_Z_TILED), with tiled=8 the [ceil(P/8), N, 8] (SLM_Z_TILED8), with
    tiled="bf16" the same in bfloat16 (SLM_Z_TILED8_BF16).
    (X, W) dtypes: (float32, float32), (bfloat16, bfloat16) or (bfloat16, float32)."""
    load()
    xt = _xdtype(X)
    wt = _xdtype(W)
    _dev(X, X.dtype, "X")
    _dev(W, W.dtype, "W")
    _dev(row_off, torch.int64, "row_off")
    N, D = X.shape
    nn = row_off.numel() - 1
    w, zb = _tile_width(tiled)
    zdt = torch.bfloat16 if zb else torch.float32
    if w:
        Z = torch.empty(((P + w - 1) // w, N, w), dtype=zdt, device=X.device)
    else:
        Z = torch.empty((N, P), dtype=torch.float32, device=X.device)
    zmin = torch.empty(nn * P, dtype=torch.float32, device=X.device)
    zmax = torch.empty_like(zmin)
    zl = Z_TILED8_BF16 if zb else {0: Z_ROWS, 32: Z_TILED, 8: Z_TILED8}[w]
    _check(_lib.slm_project(_p(X), xt, N, D, _p(W), wt, _p(row_off), nn, P, _p(Z), zl,
                            _p(zmin), _p(zmax), _stream()),
           "slm_project")
    return Z, zmin, zmax


def tile_z(Z, P: int, w: int = 32):
    """[N, P] -> particle-tiled [ceil(P/w), N, w] (padding columns zero)."""
    N = Z.shape[0]
    T = (P + w - 1) // w
    out = Z.new_zeros((N, T * w))
    out[:, :P] = Z
    return out.view(N, T, w).permute(1, 0, 2).contiguous()


def untile_z(Zt, P: int):
    """Particle-tiled [ceil(P/w), N, w] -> [N, P]."""
    T, N, w = Zt.shape
    return Zt.permute(1, 0, 2).reshape(N, T * w)[:, :P].contiguous()


# ------------------------------------------------------------------ split scan
_ws_cache: dict = {}


def scan_workspace(nbytes: int, device) -> torch.Tensor:
    """A zero-filled scratch buffer reused across calls (each call leaves it
    zero-filled again)."""
    key = (str(device),)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def split_scan(Z, zmin, zmax, target, K: int, row_off, P: int, bins: int, crit: int,
               hist: bool = False, sums: bool = False):
    """Best threshold per (node, particle); see slm_split_scan.  Z is [N, P]
    or particle-tiled [ceil(P/w), N, w] with w = 32 or 8 (float32), or
    [ceil(P/8), N, 8] bfloat16."""
    load()
    zb = Z.dtype == torch.bfloat16 and Z.dim() == 3
    _dev(Z, torch.bfloat16 if zb else torch.float32, "Z")
    _dev(row_off, torch.int64, "row_off")
    if Z.dim() == 3:
        w = Z.shape[2]
        if w not in (8, 32) or Z.shape[0] != (P + w - 1) // w or (zb and w != 8):
            raise ValueError("tiled Z must be [ceil(P/w), N, w], w = 32 or 8 (bfloat16: 8)")
        N, zl = Z.shape[1], (Z_TILED8_BF16 if zb else Z_TILED if w == 32 else Z_TILED8)
    else:
        if Z.dim() != 2 or Z.shape[1] != P:
            raise ValueError("Z must be [N, P]")
        N, zl = Z.shape[0], Z_ROWS
    nn = row_off.numel() - 1
    if crit == MSE:
        _dev(target, torch.float64, "target")
        tt = F64
    else:
        _dev(target, torch.int32, "target")
        tt = I32
    dev = Z.device
    split = torch.empty(nn * P, dtype=torch.int32, device=dev)
    loss = torch.empty(nn * P, dtype=torch.float64, device=dev)
    thr = torch.empty(nn * P, dtype=torch.float32, device=dev)
    kk = max(K, 1)
    hist_t = torch.empty(nn * P * bins * kk, dtype=torch.int32, device=dev) if (hist and bins) else None
    sums_t = torch.empty(nn * P * bins * 2, dtype=torch.float64, device=dev) if (sums and bins) else None
    need = _lib.slm_split_scan_workspace(N, nn, P, bins, K, crit)
    ws = scan_workspace(need, dev)
    _check(_lib.slm_split_scan(_p(Z), zl, _p(zmin) if bins else None, _p(zmax) if bins else None,
                               _p(target), tt, K, N, _p(row_off), nn, P, bins, crit, _p(split),
                               _p(loss), _p(thr), _p(hist_t), _p(sums_t), _p(ws), ws.numel(),
                               _stream()), "slm_split_scan")
    out = dict(split=split, loss=loss, thr=thr)
    if hist_t is not None:
        out["counts"] = hist_t.view(nn * P, bins, kk) if crit != MSE else hist_t.view(nn * P, bins)
    if sums_t is not None:
        out["sums"] = sums_t.view(nn * P, bins, 2)
    return out


def evaluate(X, W, row_off, labels, K: int, P: int, bins: int, crit: int):
    """Fused projection + histogram scan (float32, D <= 64, 2 <= K <= 4, Gini or
    entropy): zmin, zmax, split, loss, thr as slm_project + slm_split_scan."""
    load()
    _dev(X, torch.float32, "X")
    _dev(W, torch.float32, "W")
    _dev(row_off, torch.int64, "row_off")
    _dev(labels, torch.int32, "labels")
    N, D = X.shape
    nn = row_off.numel() - 1
    dev = X.device
    out = dict(zmin=torch.empty(nn * P, dtype=torch.float32, device=dev),
               zmax=torch.empty(nn * P, dtype=torch.float32, device=dev),
               split=torch.empty(nn * P, dtype=torch.int32, device=dev),
               loss=torch.empty(nn * P, dtype=torch.float64, device=dev),
               thr=torch.empty(nn * P, dtype=torch.float32, device=dev))
    need = _lib.slm_split_scan_workspace(N, nn, P, bins, K, crit)
    ws = scan_workspace(need, dev)
    _check(_lib.slm_evaluate(_p(X), N, D, _p(W), _p(row_off), nn, P, _p(labels), K, bins, crit,
                             _p(out["zmin"]), _p(out["zmax"]), _p(out["split"]), _p(out["loss"]),
                             _p(out["thr"]), _p(ws), ws.numel(), _stream()), "slm_evaluate")
    return out


# ------------------------------------------------------------------ swarm
@dataclass
class Swarm:
    x: torch.Tensor
    v: torch.Tensor
    pbest: torch.Tensor
    pbest_loss: torch.Tensor
    gbest: torch.Tensor
    gbest_loss: torch.Tensor
    gbest_p: torch.Tensor
    gbest_split: torch.Tensor
    gbest_thr: torch.Tensor
    W: torch.Tensor
    node_id: torch.Tensor
    P: int
    D: int


def pso_alloc(n_nodes: int, P: int, D: int, node_id, w_dtype=torch.float32, device="cuda"):
    f = dict(dtype=torch.float64, device=device)
    return Swarm(x=torch.empty(n_nodes * P, D, **f), v=torch.empty(n_nodes * P, D, **f),
                 pbest=torch.empty(n_nodes * P, D, **f), pbest_loss=torch.empty(n_nodes * P, **f),
                 gbest=torch.empty(n_nodes, D, **f), gbest_loss=torch.empty(n_nodes, **f),
                 gbest_p=torch.empty(n_nodes, dtype=torch.int32, device=device),
                 gbest_split=torch.full((n_nodes,), -1, dtype=torch.int32, device=device),
                 gbest_thr=torch.full((n_nodes,), float("inf"), dtype=torch.float32, device=device),
                 W=torch.empty(n_nodes * P, D, dtype=w_dtype, device=device),
                 node_id=torch.as_tensor(node_id, dtype=torch.int32).to(device).contiguous(),
                 P=P, D=D)


def pso_init(sw: Swarm, seed: int, tree: int, sel=None):
    """Initial swarm of every node; with sel (device int32 [n_nodes, n]) each
    node's swarm starts in the span of its listed dimensions
    (slm_pso_init_subspace)."""
    load()
    nn = sw.node_id.numel()
    wt = BF16 if sw.W.dtype == torch.bfloat16 else F32
    if sel is None:
        _check(_lib.slm_pso_init(_p(sw.x), _p(sw.v), _p(sw.pbest), _p(sw.pbest_loss),
                                 _p(sw.gbest), _p(sw.gbest_loss), _p(sw.gbest_p), _p(sw.node_id),
                                 nn, sw.P, sw.D, seed, tree, _p(sw.W), wt, _stream()),
               "slm_pso_init")
        return
    _dev(sel, torch.int32, "sel")
    if sel.dim() != 2 or sel.shape[0] != nn:
        raise ValueError("sel must be [n_nodes, n]")
    _check(_lib.slm_pso_init_subspace(_p(sw.x), _p(sw.v), _p(sw.pbest), _p(sw.pbest_loss),
                                      _p(sw.gbest), _p(sw.gbest_loss), _p(sw.gbest_p),
                                      _p(sw.node_id), nn, sw.P, sw.D, seed, tree, _p(sw.W), wt,
                                      _p(sel), sel.shape[1], _stream()), "slm_pso_init_subspace")


def ps_tables(R: int, alpha0: float, device="cuda"):
    """Probabilistic-search tables over R ranks (slm_ps_tables): device
    (pd float64 [R], amax int32 [R])."""
    load()
    pd = torch.empty(R, dtype=torch.float64, device=device)
    amax = torch.empty(R, dtype=torch.int32, device=device)
    _check(_lib.slm_ps_tables(int(R), float(alpha0), _p(pd), _p(amax), _stream()), "slm_ps_tables")
    return pd, amax


def ps_candidates(sw: "Swarm", ranks, pd, amax, seed: int, tree: int, t: int):
    """Candidates of the probabilistic search, iteration t, into sw.x / sw.W
    (slm_ps_candidates); ranks: device int32 [n_nodes, R]."""
    load()
    _dev(ranks, torch.int32, "ranks")
    _dev(pd, torch.float64, "pd")
    _dev(amax, torch.int32, "amax")
    nn = sw.node_id.numel()
    wt = BF16 if sw.W.dtype == torch.bfloat16 else F32
    _check(_lib.slm_ps_candidates(_p(sw.x), _p(sw.W), wt, _p(sw.node_id), nn, sw.P, sw.D,
                                  _p(ranks), ranks.shape[1], _p(pd), _p(amax), seed, tree, t,
                                  _stream()), "slm_ps_candidates")


def dft_select(X, target, K: int, row_off, bins: int, crit: int, n: int):
    """Discriminant feature test of every node and its top n channels
    (slm_dft_select): (dft_loss float64 [n_nodes, D], sel int32 [n_nodes, n])."""
    load()
    _dev(X, torch.float32, "X")
    _dev(row_off, torch.int64, "row_off")
    N, D = X.shape
    nn = row_off.numel() - 1
    if crit == MSE:
        _dev(target, torch.float64, "target")
        tt = F64
    else:
        _dev(target, torch.int32, "target")
        tt = I32
    loss = torch.empty(nn, D, dtype=torch.float64, device=X.device)
    sel = torch.empty(nn, n, dtype=torch.int32, device=X.device)
    ws = scan_workspace(_lib.slm_dft_select_workspace(N, D, nn, bins, K, crit), X.device)
    _check(_lib.slm_dft_select(_p(X), N, D, _p(row_off), nn, _p(target), tt, K, bins, crit, n,
                               _p(loss), _p(sel), _p(ws), ws.numel(), _stream()),
           "slm_dft_select")
    return loss, sel


def pso_step(sw: Swarm, loss, omega, c1, c2, seed, tree, it, move, split=None, thr=None,
             gloss=None):
    load()
    nn = sw.node_id.numel()
    wt = BF16 if sw.W.dtype == torch.bfloat16 else F32
    _dev(loss, torch.float64, "loss")
    if gloss is not None:
        _dev(gloss, torch.float64, "gloss")
    _check(_lib.slm_pso_step(_p(sw.x), _p(sw.v), _p(sw.pbest), _p(sw.pbest_loss), _p(sw.gbest),
                             _p(sw.gbest_loss), _p(sw.gbest_p), _p(loss), _p(gloss), _p(split),
                             _p(thr),
                             _p(sw.gbest_split) if split is not None else None,
                             _p(sw.gbest_thr) if thr is not None else None,
                             _p(sw.node_id), nn, sw.P, sw.D, omega, c1, c2, seed, tree, it,
                             int(bool(move)), _p(sw.W), wt, _stream()), "slm_pso_step")


@dataclass
class ApsoState:
    state: torch.Tensor     # [n] int32, 1..4
    par: torch.Tensor       # [n, 3] f64: omega, c1, c2
    dist: torch.Tensor      # [n * P] f64
    f: torch.Tensor         # [n] f64
    worst: torch.Tensor     # [n] int32
    elite: torch.Tensor     # [n, D] f64
    ws: torch.Tensor


def apso_alloc(sw: Swarm) -> ApsoState:
    """Adaptive-swarm state of every node of sw, at its start (exploration,
    omega 0.9, c1 = c2 = 2)."""
    load()
    n, dev = sw.node_id.numel(), sw.x.device
    par = torch.tensor([[0.9, 2.0, 2.0]], dtype=torch.float64, device=dev).repeat(n, 1)
    ws = torch.empty(_lib.slm_apso_workspace(n, sw.P), dtype=torch.uint8, device=dev)
    return ApsoState(state=torch.ones(n, dtype=torch.int32, device=dev), par=par,
                     dist=torch.zeros(n * sw.P, dtype=torch.float64, device=dev),
                     f=torch.zeros(n, dtype=torch.float64, device=dev),
                     worst=torch.zeros(n, dtype=torch.int32, device=dev),
                     elite=torch.zeros(n, sw.D, dtype=torch.float64, device=dev), ws=ws)


def apso_step(sw: Swarm, ap: ApsoState, loss, seed: int, tree: int, it: int, T: int, sel=None):
    """One adaptive-swarm step (bests, state estimation, move) of every node;
    sel (device int32 [n_nodes, n]): the channels each swarm lives in."""
    load()
    nn = sw.node_id.numel()
    wt = BF16 if sw.W.dtype == torch.bfloat16 else F32
    _dev(loss, torch.float64, "loss")
    n_sel = 0
    if sel is not None:
        _dev(sel, torch.int32, "sel")
        n_sel = sel.shape[-1]
    _check(_lib.slm_apso_step(_p(sw.x), _p(sw.v), _p(sw.pbest), _p(sw.pbest_loss), _p(sw.gbest),
                              _p(sw.gbest_loss), _p(sw.gbest_p), _p(loss), _p(sw.node_id), nn,
                              sw.P, sw.D, seed, tree, it, T, _p(ap.state), _p(ap.par),
                              _p(ap.dist), _p(ap.f), _p(ap.worst), _p(ap.elite), _p(sel), n_sel,
                              _p(ap.ws), ap.ws.numel(), _p(sw.W), wt, _stream()), "slm_apso_step")


# ------------------------------------------------------------------ screening
def screen_select(loss, n_nodes: int, P: int, k: int):
    """Per node the k particles with the smallest losses, ascending by
    (loss, index): int32 [n_nodes * k]."""
    load()
    _dev(loss, torch.float64, "loss")
    sel = torch.empty(n_nodes * k, dtype=torch.int32, device=loss.device)
    _check(_lib.slm_screen_select(_p(loss), n_nodes, P, k, _p(sel), _stream()),
           "slm_screen_select")
    return sel


def screen_gather(x, sel, n_nodes: int, P: int, k: int):
    """float32 images of the selected positions: [n_nodes * k, D]."""
    load()
    _dev(x, torch.float64, "x")
    _dev(sel, torch.int32, "sel")
    D = x.shape[1]
    W32 = torch.empty(n_nodes * k, D, dtype=torch.float32, device=x.device)
    _check(_lib.slm_screen_gather(_p(x), _p(sel), n_nodes, P, k, D, _p(W32), _stream()),
           "slm_screen_gather")
    return W32


def screen_merge(sel, loss_r, split_r, thr_r, n_nodes: int, P: int, k: int, loss, split, thr):
    """Re-scored results over the screened ones (in place on loss/split/thr);
    returns gloss [n_nodes * P] (re-scored loss or +inf)."""
    load()
    for t, dt, nm in ((sel, torch.int32, "sel"), (loss_r, torch.float64, "loss_r"),
                      (split_r, torch.int32, "split_r"), (thr_r, torch.float32, "thr_r"),
                      (loss, torch.float64, "loss"), (split, torch.int32, "split"),
                      (thr, torch.float32, "thr")):
        _dev(t, dt, nm)
    gloss = torch.empty(n_nodes * P, dtype=torch.float64, device=loss.device)
    _check(_lib.slm_screen_merge(_p(sel), _p(loss_r), _p(split_r), _p(thr_r), n_nodes, P, k,
                                 _p(loss), _p(split), _p(thr), _p(gloss), _stream()),
           "slm_screen_merge")
    return gloss


# ------------------------------------------------------------------ launch plans
def autotune(mode: int, path: str = None):
    """Launch plans of tree builds (slm_autotune_set): 0 = fitted rules,
    1 = cached measured plans (from path, or the file beside the library),
    2 = also measure missing shapes during tree builds and write them to
    path.  Returns the number of cached plans."""
    load()
    _check(_lib.slm_autotune_set(int(mode), path.encode() if path else None), "slm_autotune_set")
    return int(_lib.slm_autotune_plans())


# ------------------------------------------------------------------ tree
@dataclass
class TreeConfig:
    crit: int = ENTROPY
    K: int = 3
    max_depth: int = 8
    min_node: int = 32
    P: int = 256
    T: int = 50
    bins: int = 256
    omega: float = 0.7
    c1: float = 1.5
    c2: float = 1.5
    seed: int = 0
    tree: int = 0
    use_graph: bool = False
    profile: bool = False
    precision: int = 0          # 1 = bfloat16 screen, float32 re-scoring (X bfloat16)
    rescore_k: int = 32
    proposal: int = 0           # 1 = learned start from `mlp` (a device float32 tensor)
    n_seeds: int = 64
    mlp_hidden: int = 256
    mlp: object = None
    dft_top_n: int = 0          # 1..D-1: swarm in each node's top n DFT channels
    ps_R: int = 8               # proposal 2: ranks combined by the probabilistic search
    ps_alpha0: float = 10.0     # proposal 2: coefficient range of rank 1
    apso: bool = False          # adaptive swarm (APSO) in place of the plain one

    def c_params(self) -> TreeParams:
        mlp = None
        if self.proposal == 1:
            _dev(self.mlp, torch.float32, "mlp")
            mlp = self.mlp.data_ptr()
        pd = amax = None
        if self.proposal == 2:
            key = (self.ps_R, self.ps_alpha0)
            if getattr(self, "_ps_key", None) != key:
                self._ps_tables = ps_tables(self.ps_R, self.ps_alpha0)   # kept alive here
                self._ps_key = key
            pd, amax = (t.data_ptr() for t in self._ps_tables)
        return TreeParams(self.crit, self.K, self.max_depth, self.min_node, self.P, self.T,
                          self.bins, self.precision, self.rescore_k, self.omega, self.c1,
                          self.c2, self.seed, self.tree, int(self.use_graph), int(self.profile),
                          int(self.proposal), self.n_seeds, self.mlp_hidden, mlp,
                          int(self.dft_top_n), pd, amax, int(self.ps_R), int(self.apso))


_tree_ws: dict = {}


def tree_workspace(cfg: TreeConfig, N: int, D: int, device) -> torch.Tensor:
    load()
    prm = cfg.c_params()
    need = _lib.slm_grow_tree_workspace(ctypes.byref(prm), N, D)
    if need == 0:
        raise SlmError(1, "slm_grow_tree_workspace", _lib.slm_last_error().decode())
    key = str(device)
    buf = _tree_ws.get(key)
    if buf is None or buf.numel() < need:
        _tree_ws.pop(key, None)
        buf = torch.empty(need, dtype=torch.uint8, device=device)
        _tree_ws[key] = buf
    return buf


def grow_tree(X, target, cfg: TreeConfig, workspace=None, stats: bool = False):
    """One tree (Alg. 2); returns host numpy arrays of the nodes.  X is
    float32, or bfloat16 with cfg.precision = 1.  stats=True also returns each
    searched node's statistics ("stats", "sigma"; classification)."""
    load()
    _dev(X, torch.bfloat16 if cfg.precision == 1 else torch.float32, "X")
    N, D = X.shape
    if cfg.crit == MSE:
        _dev(target, torch.float64, "target")
        tt = F64
    else:
        _dev(target, torch.int32, "target")
        tt = I32
    ws = workspace if workspace is not None else tree_workspace(cfg, N, D, X.device)
    arr, out = _tree_arrays(_max_nodes(cfg, N), D, cfg.K, stats)
    prm = cfg.c_params()
    _check(_lib.slm_grow_tree(_p(X), _xdtype(X), N, D, _p(target), tt, ctypes.byref(prm), _p(ws),
                              ws.numel(), ctypes.byref(out), _stream()), "slm_grow_tree")
    return _tree_result(arr, out, cfg.K)


def _max_nodes(cfg, N: int) -> int:
    """Node capacity of one tree: 2^(max_depth+1) - 1, at most 2N + 1."""
    return int(min(2 ** (cfg.max_depth + 1) - 1, 2 * max(1, N) + 1))


def _tree_arrays(maxn: int, D: int, K: int, stats: bool = False):
    """Host output arrays of maxn nodes and the slm_tree_out that points at them."""
    kk = max(K, 1)
    arr = dict(w=np.zeros((maxn, D), np.float32), thr=np.zeros(maxn, np.float32),
               left=np.zeros(maxn, np.int32), right=np.zeros(maxn, np.int32),
               leaf=np.zeros((maxn, kk), np.float64), n=np.zeros(maxn, np.int64),
               impurity=np.zeros(maxn), split_loss=np.zeros(maxn),
               depth=np.zeros(maxn, np.int32), heap=np.zeros(maxn, np.int32),
               timing=np.zeros(TIMING_SLOTS), sample_splits=np.zeros(2, np.int64))
    if stats:
        arr["stats"] = np.zeros((maxn, (K + 1) * D), np.float32)
        arr["sigma"] = np.zeros((maxn, D), np.float32)
    out = TreeOut(maxn, 0, *[arr[k].ctypes.data for k in
                             ("w", "thr", "left", "right", "leaf", "n", "impurity", "split_loss",
                              "depth", "heap", "timing", "sample_splits")],
                  arr["stats"].ctypes.data if stats else None,
                  arr["sigma"].ctypes.data if stats else None)
    return arr, out


_NODE_FIELDS = ("w", "thr", "left", "right", "leaf", "n", "impurity", "split_loss", "depth",
                "heap", "stats", "sigma")


def _tree_result(arr, out, K):
    n = out.n_nodes
    res = {k: (v[:n] if k not in ("timing", "sample_splits") else v) for k, v in arr.items()}
    res["n_nodes"] = n
    res["K"] = K
    return res


# ------------------------------------------------------------------ ensembles
_forest_ws: dict = {}


def _cached_ws(cache: dict, need: int, device) -> torch.Tensor:
    key = str(device)
    buf = cache.get(key)
    if buf is None or buf.numel() < need:
        cache.pop(key, None)
        buf = torch.empty(need, dtype=torch.uint8, device=device)
        cache[key] = buf
    return buf


def grow_forest(X, target, cfg: TreeConfig, n_trees: int, bootstrap: bool = True,
                return_samples: bool = False):
    """SLM/SLR Forest: n_trees trees grown together, tree b on bootstrap sample
    b (tree id cfg.tree + b).  Returns the forest's host arrays (nodes of all
    trees, breadth first over the forest, roots 0 .. n_trees-1) with "tree_of"
    and "roots"; with return_samples also the drawn rows [n_trees, N]."""
    load()
    _dev(X, torch.bfloat16 if cfg.precision == 1 else torch.float32, "X")
    N, D = X.shape
    if cfg.crit == MSE:
        _dev(target, torch.float64, "target")
        tt = F64
    else:
        _dev(target, torch.int32, "target")
        tt = I32
    prm = cfg.c_params()
    need = _lib.slm_grow_forest_workspace(ctypes.byref(prm), N, D, n_trees)
    if need == 0:
        raise SlmError(1, "slm_grow_forest_workspace", _lib.slm_last_error().decode())
    ws = _cached_ws(_forest_ws, need, X.device)
    maxn = n_trees * _max_nodes(cfg, N)
    arr, out = _tree_arrays(maxn, D, cfg.K)
    tree_of = np.zeros(maxn, np.int32)
    samples = (torch.empty((n_trees, N), dtype=torch.int32, device=X.device)
               if return_samples and bootstrap else None)
    _check(_lib.slm_grow_forest(_p(X), _xdtype(X), N, D, _p(target), tt, ctypes.byref(prm),
                                n_trees, int(bootstrap), _p(ws), ws.numel(), _p(samples),
                                ctypes.byref(out), tree_of.ctypes.data, _stream()),
           "slm_grow_forest")
    res = _tree_result(arr, out, cfg.K)
    res["tree_of"] = tree_of[:out.n_nodes]
    res["roots"] = np.arange(n_trees, dtype=np.int32)
    res["n_trees"] = n_trees
    if return_samples:
        res["samples"] = samples
    return res


def forest_tree(forest: dict, b: int) -> dict:
    """Tree b of a forest as a stand-alone tree dict (nodes renumbered from 0 in
    forest order, which is the tree's own breadth-first order)."""
    idx = np.nonzero(forest["tree_of"] == b)[0]
    remap = np.full(forest["n_nodes"], -1, np.int64)
    remap[idx] = np.arange(idx.size)
    res = {k: forest[k][idx].copy() for k in _NODE_FIELDS if k in forest}
    for k in ("left", "right"):
        c = res[k]
        res[k] = np.where(c >= 0, remap[np.maximum(c, 0)], -1).astype(np.int32)
    res["n_nodes"] = idx.size
    res["K"] = forest["K"]
    return res


def forest_predict(forest: dict, X, return_leaves: bool = False):
    """Forest output for the rows X (device float32): majority class (int32)
    or mean (float64); return_leaves also gives the leaf ids [n_trees, N]."""
    load()
    _dev(X, torch.float32, "X")
    dev = X.device
    t = {k: torch.from_numpy(np.ascontiguousarray(forest[k])).to(dev)
         for k in ("w", "thr", "left", "right", "leaf", "roots")}
    nt = int(forest["roots"].size)
    N, D = X.shape
    leaves = torch.empty((nt, N), dtype=torch.int32, device=dev)
    K = forest["K"] if forest["K"] > 1 else 0
    out = torch.empty(N, dtype=torch.int32 if K else torch.float64, device=dev)
    _check(_lib.slm_forest_predict(_p(t["w"]), _p(t["thr"]), _p(t["left"]), _p(t["right"]),
                                   _p(t["leaf"]), int(forest["n_nodes"]), _p(t["roots"]), nt, D, K,
                                   _p(X), N, _p(leaves), _p(out), _stream()), "slm_forest_predict")
    return (out, leaves) if return_leaves else out


_boost_ws: dict = {}


def boost(X, target, cfg: TreeConfig, n_rounds: int, lr: float, n_classes: int = 0):
    """SLM/SLR Boost: n_rounds rounds of SLR trees (cfg must be an MSE config)
    on negative gradients; n_classes = 0 for regression (target float64),
    else K-class softmax (target int32 labels).  Returns host arrays of all
    trees (round order) with "tree_of", "F0", the learning rate and the final
    training scores F (device [N, max(K, 1)])."""
    load()
    _dev(X, torch.float32, "X")
    N, D = X.shape
    if n_classes:
        _dev(target, torch.int32, "target")
        tt = I32
    else:
        _dev(target, torch.float64, "target")
        tt = F64
    prm = cfg.c_params()
    need = _lib.slm_boost_workspace(ctypes.byref(prm), N, D, n_classes)
    if need == 0:
        raise SlmError(1, "slm_boost_workspace", _lib.slm_last_error().decode())
    ws = _cached_ws(_boost_ws, need, X.device)
    Kc = max(1, n_classes)
    maxn = max(1, n_rounds * Kc * _max_nodes(cfg, N))
    arr, out = _tree_arrays(maxn, D, 0)
    tree_of = np.zeros(maxn, np.int32)
    F = torch.empty((N, Kc), dtype=torch.float64, device=X.device)
    F0 = np.zeros(Kc)
    _check(_lib.slm_boost(_p(X), N, D, _p(target), tt, n_classes, ctypes.byref(prm), n_rounds,
                          float(lr), _p(ws), ws.numel(), _p(F), F0.ctypes.data,
                          ctypes.byref(out), tree_of.ctypes.data, _stream()), "slm_boost")
    res = _tree_result(arr, out, 0)
    res["tree_of"] = tree_of[:out.n_nodes]
    res.update(F0=F0, lr=float(lr), n_classes=n_classes, n_rounds=n_rounds, F=F)
    return res


def boost_scores(model: dict, X, rounds=None):
    """F(x) of a boosted model on the device (slm_boost_scores): F0 + lr *
    the trees' leaf values, added round by round ([N, max(K, 1)] float64);
    rounds limits the sum to the first rounds."""
    load()
    _dev(X, torch.float32, "X")
    Kc = max(1, model["n_classes"])
    N, D = X.shape
    n_rounds = model["n_rounds"] if rounds is None else rounds
    nt = n_rounds * Kc
    dev = X.device
    roots = np.array([np.nonzero(model["tree_of"] == t)[0][0] for t in range(nt)], dtype=np.int32)
    t = {k: torch.from_numpy(np.ascontiguousarray(model[k])).to(dev)
         for k in ("w", "thr", "left", "right", "leaf")}
    r = torch.from_numpy(roots).to(dev)
    leaves = torch.empty((max(1, nt), N), dtype=torch.int32, device=dev)
    F = torch.empty((N, Kc), dtype=torch.float64, device=dev)
    F0 = np.ascontiguousarray(model["F0"], dtype=np.float64)
    _check(_lib.slm_boost_scores(_p(t["w"]), _p(t["thr"]), _p(t["left"]), _p(t["right"]),
                                 _p(t["leaf"]), int(model["n_nodes"]), _p(r), int(n_rounds),
                                 int(model["n_classes"]), D, F0.ctypes.data, float(model["lr"]),
                                 _p(X), N, _p(leaves), _p(F), _stream()), "slm_boost_scores")
    return F


# ------------------------------------------------------------------ node-batch search
def search_nodes(X, target, row_off, node_id, cfg: TreeConfig, target_loss=None, workspace=None):
    """Swarm search of a batch of nodes (rows grouped by node, row_off int64
    [n+1] on the device); optional per-node stop targets.  Returns device
    tensors gbest [n, D], gbest_loss, gbest_split, gbest_thr, evals."""
    load()
    _dev(X, torch.bfloat16 if cfg.precision == 1 else torch.float32, "X")
    _dev(row_off, torch.int64, "row_off")
    _dev(node_id, torch.int32, "node_id")
    N, D = X.shape
    nn = row_off.numel() - 1
    if cfg.crit == MSE:
        _dev(target, torch.float64, "target")
        tt = F64
    else:
        _dev(target, torch.int32, "target")
        tt = I32
    if target_loss is not None:
        _dev(target_loss, torch.float64, "target_loss")
    prm = cfg.c_params()
    need = _lib.slm_search_nodes_workspace(ctypes.byref(prm), N, D, nn)
    if need == 0:
        raise SlmError(1, "slm_search_nodes_workspace", _lib.slm_last_error().decode())
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=X.device)
    dev = X.device
    out = dict(gbest=torch.empty(nn, D, dtype=torch.float64, device=dev),
               gbest_loss=torch.empty(nn, dtype=torch.float64, device=dev),
               gbest_split=torch.empty(nn, dtype=torch.int32, device=dev),
               gbest_thr=torch.empty(nn, dtype=torch.float32, device=dev),
               evals=torch.empty(nn, dtype=torch.int32, device=dev))
    _check(_lib.slm_search_nodes(_p(X), _xdtype(X), N, D, _p(target), tt, _p(row_off),
                                 _p(node_id), nn, ctypes.byref(prm), _p(target_loss),
                                 _p(out["gbest"]), _p(out["gbest_loss"]), _p(out["gbest_split"]),
                                 _p(out["gbest_thr"]), _p(out["evals"]), _p(workspace),
                                 workspace.numel(), _stream()), "slm_search_nodes")
    return out


# ------------------------------------------------------------------ learned proposal
def node_stats(X, labels, K: int, row_off):
    """Per-node statistics [n, (K+1) D] and deviations [n, D] (float32)."""
    load()
    _dev(X, X.dtype, "X")
    _dev(labels, torch.int32, "labels")
    _dev(row_off, torch.int64, "row_off")
    N, D = X.shape
    nn = row_off.numel() - 1
    stats = torch.empty(nn, (K + 1) * D, dtype=torch.float32, device=X.device)
    sigma = torch.empty(nn, D, dtype=torch.float32, device=X.device)
    need = _lib.slm_node_stats_workspace(nn, D, K)
    ws = torch.zeros(need, dtype=torch.uint8, device=X.device)
    _check(_lib.slm_node_stats(_p(X), _xdtype(X), N, D, _p(labels), K, _p(row_off), nn,
                               _p(stats), _p(sigma), _p(ws), ws.numel(), _stream()),
           "slm_node_stats")
    return stats, sigma


def mlp_param_count(n_in: int, hidden: int, n_out: int) -> int:
    load()
    return int(_lib.slm_mlp_param_count(n_in, hidden, n_out))


def mlp_forward(params, n_in: int, hidden: int, n_out: int, inp, bf16: bool = False):
    """(out [B, n_out], cache [4, B, hidden]: z1, h1, z2, h2)."""
    load()
    _dev(params, torch.float32, "params")
    _dev(inp, torch.float32, "in")
    B = inp.shape[0]
    out = torch.empty(B, n_out, dtype=torch.float32, device=inp.device)
    cache = torch.empty(4, B, hidden, dtype=torch.float32, device=inp.device)
    _check(_lib.slm_mlp_forward(_p(params), n_in, hidden, n_out, _p(inp), B, int(bool(bf16)),
                                _p(out), _p(cache), _stream()), "slm_mlp_forward")
    return out, cache


def mlp_backward(params, n_in: int, hidden: int, n_out: int, inp, cache, d_out):
    load()
    for t, nm in ((params, "params"), (inp, "in"), (cache, "cache"), (d_out, "d_out")):
        _dev(t, torch.float32, nm)
    B = inp.shape[0]
    grads = torch.empty_like(params)
    work = torch.empty(B, 2 * hidden, dtype=torch.float32, device=inp.device)
    _check(_lib.slm_mlp_backward(_p(params), n_in, hidden, n_out, _p(inp), B, _p(cache),
                                 _p(d_out), _p(grads), _p(work), _stream()), "slm_mlp_backward")
    return grads


def wta_loss(out, target, M: int, eps: float, scale: float = 1.0):
    """(loss [B], scale * d_out [B, M D]) of the relaxed winner-take-all loss."""
    load()
    _dev(out, torch.float32, "out")
    _dev(target, torch.float32, "target")
    B, D = target.shape
    loss = torch.empty(B, dtype=torch.float32, device=out.device)
    d_out = torch.empty_like(out)
    _check(_lib.slm_wta_loss(_p(out), _p(target), B, M, D, float(eps), float(scale), _p(loss),
                             _p(d_out), _stream()), "slm_wta_loss")
    return loss, d_out


def proposal_targets(g, sigma):
    """Standardised unit targets t = g sigma / |g sigma| ([n, D] float32)."""
    load()
    _dev(g, torch.float32, "g")
    _dev(sigma, torch.float32, "sigma")
    n, D = g.shape
    t = torch.empty_like(g)
    _check(_lib.slm_proposal_targets(_p(g), _p(sigma), n, D, _p(t), _stream()),
           "slm_proposal_targets")
    return t


def adam_step(params, grads, m, v, lr: float, step: int, b1=0.9, b2=0.999, eps=1e-8):
    load()
    for t, nm in ((params, "params"), (grads, "grads"), (m, "m"), (v, "v")):
        _dev(t, torch.float32, nm)
    _check(_lib.slm_adam_step(_p(params), _p(grads), _p(m), _p(v), params.numel(), float(lr),
                              float(b1), float(b2), float(eps), int(step), _stream()),
           "slm_adam_step")


def proposal_seeds(out, sigma, M: int, sw: "Swarm"):
    """Write the network's seeds into the first min(M, P) particles of sw."""
    load()
    _dev(out, torch.float32, "out")
    _dev(sigma, torch.float32, "sigma")
    nn = sigma.shape[0]
    wt = BF16 if sw.W.dtype == torch.bfloat16 else F32
    _check(_lib.slm_proposal_seeds(_p(out), _p(sigma), nn, M, sw.D, sw.P, _p(sw.x), _p(sw.pbest),
                                   _p(sw.W), wt, _stream()), "slm_proposal_seeds")


def predict_leaves(tree: dict, X):
    """Leaf index reached by each row (right iff float32 w.x >= thr)."""
    load()
    _dev(X, torch.float32, "X")
    dev = X.device
    w = torch.from_numpy(np.ascontiguousarray(tree["w"])).to(dev)
    thr = torch.from_numpy(np.ascontiguousarray(tree["thr"])).to(dev)
    left = torch.from_numpy(np.ascontiguousarray(tree["left"])).to(dev)
    right = torch.from_numpy(np.ascontiguousarray(tree["right"])).to(dev)
    out = torch.empty(X.shape[0], dtype=torch.int32, device=dev)
    _check(_lib.slm_predict(_p(w), _p(thr), _p(left), _p(right), int(tree["n_nodes"]), X.shape[1],
                            _p(X), X.shape[0], _p(out), _stream()), "slm_predict")
    return out


def predict(tree: dict, X):
    """Class ids (the leaf's majority class, smallest on ties) or regression
    means of the rows X, computed on the device as a one-tree forest
    (slm_forest_predict); returned as a host array."""
    one = {k: tree[k] for k in ("w", "thr", "left", "right", "leaf", "n_nodes", "K")}
    one["roots"] = np.zeros(1, np.int32)
    return forest_predict(one, X).cpu().numpy()
