"""Benchmark: SLM split search on one MI355X, in projected sample-splits/s.

Headline workload (one step = one tree, the whole split-search path):
mixed-precision screening tree.  N = 4 000 000 rows, D = 256, 10 classes with
means ~N(0, I) and a shared covariance L L^T + diag(delta) of rank 16, X stored
bfloat16.  Every node's P = 1024 particles are screened with the bfloat16 MFMA
projection (FP32 accumulation) and a 256-bin histogram scan; the best 32 are
projected again with FP32 directions and re-scanned; the swarm moves T = 40
times (41 evaluations); Gini criterion; depth 12, minimum node size 32; all
frontier nodes of a depth are searched together (each depth's swarm loop
replayed as a HIP graph).  Synthetic seeded data, resident in HBM before the
timed region.

Prints one JSON line.  `value` = sum over evaluations of n_node * P (the
screened sample-splits) divided by the timed wall time; the re-scored
sample-splits (n_node * 32) are reported beside it.  `roofline` is the
dominant kernel's (the screened projection) achieved rate, from HIP events
around every launch of one extra instrumented tree.  Secondary lines: the
plain tree (N = 1e5, D = 64, K = 3), the regression tree (N = 1e6, D = 128,
MSE), the single-node latency (N = 1000, D = 8, exact scan), the learned
proposal against random starts, and the oracle's CPU rate (`cpu_baseline`).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "projected sample-splits/s; SLM tree train time, learned vs plain @ equal loss"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and, in a
# second run, WRITE_SIZE (KiB per dispatch, mean over the dispatches of the
# run), scaled by what the same counters read for a plain 1 GiB device copy
# (FETCH_SIZE 524305 KiB -> x 2.0, WRITE_SIZE 1048576 KiB -> x 1.0).  Valid
# only for the kernel source they were taken on (SHA-256 of the file);
# otherwise the traffic is reported as null.  Summaries and commands:
# profiles/traffic_*.md
TRAFFIC = {
    "k_project_stream_bf16": {
        "source": "paper_2208_07023_amd/csrc/k_project.hip",
        "sha256": "f49c983402a94fef5cc8a95bb6301aa6894bd516fe691aa361c66aabc7109614",
        "fetch_kib": 664628.5, "write_kib": 3776262.8,
        "profile": "profiles/traffic_screened_projection_N4M_D256_P1024.md",
    },
}
FETCH_SCALE, WRITE_SCALE = 1048576.0 / 524305.0, 1.0


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the stored counters, or None when
    none are stored or its source has changed since they were taken."""
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
            return None
    return (t["fetch_kib"] * FETCH_SCALE + t["write_kib"] * WRITE_SCALE) * 1024.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_info():
    """Host cores this process may use (capped at the 16 of a one-GPU share)
    and the CPU model name."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable": min(avail, 16), "model": model}


# ------------------------------------------------------------------ workloads
def screening_config(api):
    return api.TreeConfig(crit=api.GINI, K=10, max_depth=12, min_node=32, P=1024, T=40, bins=256,
                          precision=1, rescore_k=32, seed=0, use_graph=True)


def screening_data(dev):
    import torch

    from paper_2208_07023_amd import inputs
    bits, y = inputs.lowrank_mixture(4_000_000, 256, 10, rank=16, seed=0)
    Xd = torch.from_numpy(bits.view(np.int16)).to(dev).view(torch.bfloat16)
    return bits, y, Xd, torch.from_numpy(y).to(dev)


def timed_trees(api, Xd, yd, cfg, steps, warmup, ws, what):
    import torch
    for w in range(warmup):
        cfg.tree = 1000 + w
        api.grow_tree(Xd, yd, cfg, workspace=ws)
        log(f"{what}: warmup {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    trees = []
    t0 = time.perf_counter()
    for k in range(steps):
        cfg.tree = k
        trees.append(api.grow_tree(Xd, yd, cfg, workspace=ws))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ss = sum(int(t["sample_splits"][0]) for t in trees)
    ssr = sum(int(t["sample_splits"][1]) for t in trees)
    log(f"{what}: {steps} trees in {dt:.3f} s, {ss / dt:.4g} sample-splits/s, "
        f"device ms {[round(t['timing'][0], 1) for t in trees]}")
    return trees, dt, ss, ssr


def instrumented(api, Xd, yd, cfg, ws):
    """One tree without graph replay, HIP events around every launch."""
    cfg.tree = 0
    cfg.profile = True
    use_graph = cfg.use_graph
    cfg.use_graph = False
    tr = api.grow_tree(Xd, yd, cfg, workspace=ws)
    cfg.profile = False
    cfg.use_graph = use_graph
    return tr


def headline(api, args, dev):
    """The screening tree: timed trees, then one instrumented tree."""
    import torch
    t0 = time.perf_counter()
    bits, y, Xd, yd = screening_data(dev)
    log(f"screening data ready in {time.perf_counter() - t0:.1f} s")
    N, D = Xd.shape
    cfg = screening_config(api)
    ws = api.tree_workspace(cfg, N, D, dev)
    torch.cuda.synchronize()
    trees, dt, ss, ssr = timed_trees(api, Xd, yd, cfg, args.steps, args.warmup, ws, "screening tree")
    prof = instrumented(api, Xd, yd, cfg, ws)
    tm = prof["timing"]
    ss_p, ssr_p = int(prof["sample_splits"][0]), int(prof["sample_splits"][1])
    rows_p = ss_p / cfg.P                      # row-evaluations of the tree
    k = cfg.rescore_k
    # algorithmic bytes: the screened projection writes 2 B of bfloat16 Z
    # per sample-split and reads each row's 2 D bytes of X once; the scan
    # reads 2 B of Z per sample-split and each row's 4-byte label once
    proj_bytes = 2.0 * ss_p + rows_p * 2 * D
    proj_flops = 2.0 * D * ss_p
    scan_bytes = 2.0 * ss_p + 4.0 * rows_p
    rproj_flops = 2.0 * D * ssr_p
    # the re-scoring reads each row's X again and writes 4 B of float32 Z per
    # re-scored sample-split; its 2 D flops (three bfloat16 products each) per
    # 4 + 2 D / k bytes keep it below the matrix cores' ridge: HBM-bound
    rproj_bytes = 4.0 * ssr_p + rows_p * 2 * D
    rscan_bytes = 4.0 * ssr_p + 4.0 * rows_p
    n_proj, n_scan, n_rp, n_rs = (max(1, int(tm[i])) for i in (6, 7, 10, 11))
    proj_s, scan_s, rp_s, rs_s = (tm[i] * 1e-3 for i in (3, 4, 8, 9))
    proj_gbs = proj_bytes / proj_s / 1e9
    kernels = {
        "project_screened_bf16": {"kernel": "k_project_stream (BF16 MFMA)", "launches": n_proj,
                                  "avg_us": 1e6 * proj_s / n_proj,
                                  "bytes_per_launch": proj_bytes / n_proj, "GB/s": proj_gbs,
                                  "frac_hbm": proj_gbs / HBM_PEAK_GBS,
                                  "TFLOP/s": proj_flops / proj_s / 1e12,
                                  "frac_bf16_mfma": proj_flops / proj_s / 1e12 / BF16_PEAK_TFLOPS,
                                  "traffic": measured_traffic("k_project_stream_bf16")},
        "scan_screened": {"launches": n_scan, "avg_us": 1e6 * scan_s / n_scan,
                          "bytes_per_launch": scan_bytes / n_scan,
                          "GB/s": scan_bytes / scan_s / 1e9,
                          "frac_hbm": scan_bytes / scan_s / 1e9 / HBM_PEAK_GBS},
        "project_rescore_f32": {"kernel": "k_project_stream (float32 directions as three "
                                          "bfloat16 parts, BF16 MFMA)",
                                "launches": n_rp, "avg_us": 1e6 * rp_s / n_rp,
                                "bytes_per_launch": rproj_bytes / n_rp,
                                "GB/s": rproj_bytes / rp_s / 1e9,
                                "frac_hbm": rproj_bytes / rp_s / 1e9 / HBM_PEAK_GBS,
                                "TFLOP/s": rproj_flops / rp_s / 1e12},
        "scan_rescore": {"launches": n_rs, "avg_us": 1e6 * rs_s / n_rs,
                         "GB/s": rscan_bytes / rs_s / 1e9},
        "swarm_steps_ms": tm[5], "partitions_ms": tm[2], "tree_ms_instrumented": tm[0],
    }
    roof = {"bound": "hbm", "kernel": "k_project_stream<BF16> (screened projection)",
            "achieved": proj_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": proj_gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic("k_project_stream_bf16"),
            "bytes_per_launch": proj_bytes / n_proj,
            "note": "algorithmic bytes: 2 B of bfloat16 Z written per sample-split + 2 D B "
                    "of bfloat16 X read per row; 2 D flops per 2 B of Z is 256 flop/B at "
                    "D = 256, below the BF16 ridge of 312 flop/B, so the projection is "
                    "HBM-bound"}
    depths = np.bincount(trees[0]["depth"]).tolist()
    res = {
        "value": ss / dt, "ms_per_step": 1e3 * dt / args.steps, "steps": args.steps,
        "sample_splits_rescored_per_s": ssr / dt,
        "config": {"workload": "BF16 screening tree: N=4000000, D=256, K=10 (class means ~N(0,I), "
                               "shared covariance LL^T+diag, rank 16), X bfloat16; P=1024 "
                               "screened by BF16 MFMA (FP32 accumulate, projections stored "
                               "in BF16), top 32 re-scored in FP32; T=40; Gini; 256-bin "
                               "histogram; depth 12; min node 32",
                   "nodes_per_tree": float(np.mean([t["n_nodes"] for t in trees])),
                   "nodes_per_depth_tree0": depths,
                   "sample_splits_per_tree": ss // args.steps,
                   "rescored_sample_splits_per_tree": ssr // args.steps,
                   "hip_graph": True},
        "roofline": roof, "kernels": kernels,
    }
    res["screening_gpu"] = screening_gpu_check(api, Xd, yd, cfg)
    del ws
    api._tree_ws.clear()
    torch.cuda.empty_cache()
    return res, (bits, y)


def screening_gpu_check(api, Xd, yd, cfg, n_swarms=4):
    """At the root: all P particles projected in FP32 (the re-scoring
    projection with k = P) against the screened evaluation, GPU only: how
    often the FP32-best particle is among the screened top k, the relative
    gap between the best re-scored loss and the FP32 best, and the screened
    losses' relative error against the FP32 ones.  The same quantities
    against the FP64 oracle are asserted in the GPU tests."""
    import torch
    N, D = Xd.shape
    P, k = cfg.P, cfg.rescore_k
    off = torch.tensor([0, N], dtype=torch.int64, device=Xd.device)
    hits, gaps, errs = 0, [], []
    for s in range(n_swarms):
        sw = api.pso_alloc(1, P, D, node_id=[0], w_dtype=torch.bfloat16)
        api.pso_init(sw, seed=100 + s, tree=0)
        Zs, zmin, zmax = api.project(Xd, sw.W, off, P, tiled="bf16")
        scr = api.split_scan(Zs, zmin, zmax, yd, cfg.K, off, P, cfg.bins, api.GINI)
        del Zs
        sel = api.screen_select(scr["loss"], 1, P, k).cpu().numpy()
        W32 = sw.x.to(torch.float32).contiguous()
        Zf, fmin, fmax = api.project(Xd, W32, off, P, tiled=8)
        full = api.split_scan(Zf, fmin, fmax, yd, cfg.K, off, P, cfg.bins, api.GINI)
        del Zf
        lf = full["loss"].cpu().numpy()
        ls = scr["loss"].cpu().numpy()
        best = int(np.argmin(lf))
        hits += int(best in set(sel.tolist()))
        gaps.append(float((lf[sel].min() - lf[best]) / lf[best]))
        errs.append(np.abs(ls - lf) / lf)
        torch.cuda.empty_cache()
    e = np.concatenate(errs)
    return {"swarms": n_swarms, "P": P, "k": k,
            "fp32_best_in_screened_topk": hits / n_swarms,
            "rel_gap_best_rescored_vs_fp32_best": {"mean": float(np.mean(gaps)),
                                                   "max": float(np.max(gaps))},
            "screened_loss_rel_err_vs_fp32": {"median": float(np.median(e)),
                                              "p99": float(np.quantile(e, 0.99)),
                                              "max": float(e.max())}}


def plain_tree_line(api, dev, steps=5, warmup=2):
    """Plain FP32 tree: N = 1e5, D = 64, 3 classes x 4 clusters, P = 256,
    T = 50, entropy, 256 bins, depth 8, min node 32."""
    import torch

    from paper_2208_07023_amd import inputs
    N, D, K = 100_000, 64, 3
    X, y = inputs.cluster_mixture(N, D, K, clusters_per_class=4, mean_std=2.0, seed=0)
    Xd, yd = torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev)
    cfg = api.TreeConfig(crit=api.ENTROPY, K=K, max_depth=8, min_node=32, P=256, T=50, bins=256,
                         seed=0, use_graph=True)
    ws = api.tree_workspace(cfg, N, D, dev)
    trees, dt, ss, _ = timed_trees(api, Xd, yd, cfg, steps, warmup, ws, "plain tree")
    prof = instrumented(api, Xd, yd, cfg, ws)
    tm = prof["timing"]
    ss_p = int(prof["sample_splits"][0])
    rows_p = ss_p / cfg.P
    proj_tfs = 2.0 * D * ss_p / (tm[3] * 1e-3) / 1e12
    scan_gbs = (4.0 * ss_p + 4.0 * rows_p) / (tm[4] * 1e-3) / 1e9
    acc = float((api.predict(trees[0], Xd) == y).mean())
    return {"workload": f"plain SLM tree: N={N}, D={D}, K={K} (4 Gaussian clusters/class), P=256, "
                        "T=50, 256-bin histogram, entropy, depth 8, min node 32",
            "sample_splits_per_s": ss / dt, "ms_per_tree": 1e3 * dt / steps,
            "nodes_per_tree": float(np.mean([t["n_nodes"] for t in trees])),
            "train_accuracy": acc,
            "k_project_short": {"avg_us": 1e3 * tm[3] / max(1, tm[6]), "TFLOP/s": proj_tfs,
                                "frac_fp32_mfma": proj_tfs / FP32_PEAK_TFLOPS},
            "scan": {"avg_us": 1e3 * tm[4] / max(1, tm[7]), "GB/s": scan_gbs,
                     "frac_hbm": scan_gbs / HBM_PEAK_GBS}}, (X, y, Xd, yd)


def regression_tree_line(api, dev, steps=3, warmup=1):
    """Regression tree: N = 1e6, D = 128, y = sum_k |x.u_k| + noise, P = 512,
    T = 40, MSE with FP64 sums, 256 bins, depth 10, min node 32."""
    import torch

    from paper_2208_07023_amd import inputs
    N, D = 1_000_000, 128
    X, y = inputs.abs_direction_regression(N, D, seed=0)
    Xd, yd = torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev)
    cfg = api.TreeConfig(crit=api.MSE, K=0, max_depth=10, min_node=32, P=512, T=40, bins=256,
                         seed=0, use_graph=True)
    ws = api.tree_workspace(cfg, N, D, dev)
    trees, dt, ss, _ = timed_trees(api, Xd, yd, cfg, steps, warmup, ws, "regression tree")
    prof = instrumented(api, Xd, yd, cfg, ws)
    tm = prof["timing"]
    ss_p = int(prof["sample_splits"][0])
    rows_p = ss_p / cfg.P
    proj_tfs = 2.0 * D * ss_p / (tm[3] * 1e-3) / 1e12
    scan_gbs = (4.0 * ss_p + 8.0 * rows_p) / (tm[4] * 1e-3) / 1e9
    mse = float(np.mean((api.predict(trees[0], Xd) - y) ** 2))
    res = {"workload": f"SLM regression tree: N={N}, D={D}, y = sum of |x.u_k| (8 directions) + "
                       "N(0,0.1^2); P=512, T=40, MSE (FP64 sums), 256-bin histogram, depth 10, "
                       "min node 32",
           "sample_splits_per_s": ss / dt, "ms_per_tree": 1e3 * dt / steps,
           "nodes_per_tree": float(np.mean([t["n_nodes"] for t in trees])),
           "train_mse": mse, "target_var": float(np.var(y)),
           "k_project": {"avg_us": 1e3 * tm[3] / max(1, tm[6]), "TFLOP/s": proj_tfs,
                         "frac_fp32_mfma": proj_tfs / FP32_PEAK_TFLOPS},
           "scan": {"avg_us": 1e3 * tm[4] / max(1, tm[7]), "GB/s": scan_gbs,
                    "frac_hbm": scan_gbs / HBM_PEAK_GBS}}
    del ws
    api._tree_ws.clear()
    torch.cuda.empty_cache()
    return res


def single_node_line(api, dev, reps=50):
    """Single node: N = 1000, D = 8, 2 classes, P = 32, T = 20 (21
    evaluations), exact sort scan, Gini -- bound by launch latency.  The
    swarm loop is one graph replay; its HIP-event time is reported per PSO
    and per evaluation (from the difference of T = 20 and T = 0)."""
    import torch

    from paper_2208_07023_amd import inputs
    X, y, _ = inputs.two_class_gaussian(1000, 8, seed=0)
    Xd, yd = torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev)
    out = {}
    for T in (0, 20):
        cfg = api.TreeConfig(crit=api.GINI, K=2, max_depth=1, min_node=32, P=32, T=T, bins=0,
                             seed=0, use_graph=True)
        for w in range(3):
            cfg.tree = w
            api.grow_tree(Xd, yd, cfg)
        sw, tot = [], []
        for r in range(reps):
            cfg.tree = r
            t0 = time.perf_counter()
            tr = api.grow_tree(Xd, yd, cfg)
            tot.append(time.perf_counter() - t0)
            sw.append(tr["timing"][1])
        out[T] = (float(np.median(sw)) * 1e3, float(np.median(tot)) * 1e6)
    return {"workload": "single node: N=1000, D=8, 2 classes, P=32, T=20 (21 evaluations), "
                        "exact sort scan, Gini",
            "us_per_pso_21_evals": out[20][0],
            "us_per_evaluation": (out[20][0] - out[0][0]) / 20.0,
            "us_per_depth1_tree_call": out[20][1],
            "sample_splits_per_s": 21 * 1000 * 32 / (out[20][0] * 1e-6)}


def tune_plans(api, path, dev):
    """Measure the launch plans of one tree of each workload (the first
    evaluation of every depth times its shapes' candidate plans) into path."""
    import torch

    from paper_2208_07023_amd import inputs
    api.autotune(2, path)
    out = {}
    _, _, Xd, yd = screening_data(dev)
    cfg = screening_config(api)
    t0 = time.perf_counter()
    api.grow_tree(Xd, yd, cfg)
    out["screening_s"] = time.perf_counter() - t0
    del Xd, yd
    api._tree_ws.clear()
    torch.cuda.empty_cache()
    X, y = inputs.cluster_mixture(100_000, 64, 3, clusters_per_class=4, mean_std=2.0, seed=0)
    cfg = api.TreeConfig(crit=api.ENTROPY, K=3, max_depth=8, min_node=32, P=256, T=50, bins=256,
                         seed=0, use_graph=True)
    t0 = time.perf_counter()
    api.grow_tree(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), cfg)
    out["plain_s"] = time.perf_counter() - t0
    X, y = inputs.abs_direction_regression(1_000_000, 128, seed=0)
    cfg = api.TreeConfig(crit=api.MSE, K=0, max_depth=10, min_node=32, P=512, T=40, bins=256,
                         seed=0, use_graph=True)
    t0 = time.perf_counter()
    api.grow_tree(torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev), cfg)
    out["regression_s"] = time.perf_counter() - t0
    out["plans"] = api.autotune(1, path)
    out["path"] = path
    log(f"tuned plans: {out}")
    return out


def root_evals(api, which, reps, dev):
    """`reps` root evaluations of a workload through the C ABI, each timed
    with HIP events on the launch stream: the screened projection (BF16) and
    scan, the FP32 re-scoring of the best 32 (screening tree), or the FP32
    projection and scan (plain and regression trees)."""
    import torch

    from paper_2208_07023_amd import inputs
    if which == "screening":
        _, _, Xd, yd = screening_data(dev)
        K, P, crit, wdt = 10, 1024, api.GINI, torch.bfloat16
    elif which == "plain":
        X, y = inputs.cluster_mixture(100_000, 64, 3, clusters_per_class=4, mean_std=2.0, seed=0)
        Xd, yd = torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev)
        K, P, crit, wdt = 3, 256, api.ENTROPY, torch.float32
    else:
        X, y = inputs.abs_direction_regression(1_000_000, 128, seed=0)
        Xd, yd = torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev)
        K, P, crit, wdt = 0, 512, api.MSE, torch.float32
    N, D = Xd.shape
    off = torch.tensor([0, N], dtype=torch.int64, device=dev)
    sw = api.pso_alloc(1, P, D, node_id=[0], w_dtype=wdt)
    api.pso_init(sw, seed=0, tree=0)
    st = torch.cuda.current_stream()
    times = {"project": [], "scan": [], "rescore_project": [], "rescore_scan": []}

    def timed(key, fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        r = fn()
        e1.record(st)
        times[key].append((e0, e1))
        return r

    for _ in range(reps):
        # the tree's storage: bfloat16 8-wide tiles for the screening pass
        zt = "bf16" if which == "screening" else 8
        Z, zmin, zmax = timed("project", lambda: api.project(Xd, sw.W, off, P, tiled=zt))
        out = timed("scan", lambda: api.split_scan(Z, zmin, zmax, yd, K, off, P, 256, crit))
        if which == "screening":
            sel = api.screen_select(out["loss"], 1, P, 32)
            Wk = api.screen_gather(sw.x, sel, 1, P, 32)
            Zr, rmin, rmax = timed("rescore_project", lambda: api.project(Xd, Wk, off, 32,
                                                                          tiled=8))
            timed("rescore_scan", lambda: api.split_scan(Zr, rmin, rmax, yd, K, off, 32, 256,
                                                         crit))
        del Z
    torch.cuda.synchronize()
    res = {"workload": which, "N": N, "D": D, "P": P, "reps": reps}
    for k, v in times.items():
        if v:
            res[k + "_ms"] = [round(a.elapsed_time(b), 4) for a, b in v]
    return res


# ------------------------------------------------------------------ extras
def dft_vs_plain(api, Xd, yd, y, K, reps=2):
    """Swarm in each node's top n DFT channels (Alg. 2) against the swarm in
    all D dimensions, on the plain-tree data: for T = 5, 20, 50 moves, the
    root's split loss, the tree's training accuracy and the time per tree."""
    import torch
    D = Xd.shape[1]
    res = {}
    for n in (0, 16):
        arm = {}
        for T in (5, 20, 50):
            cfg = api.TreeConfig(crit=api.ENTROPY, K=K, max_depth=8, min_node=32, P=256, T=T,
                                 bins=256, seed=0, use_graph=True, dft_top_n=n)
            api.grow_tree(Xd, yd, cfg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            trees = []
            for r in range(reps):
                cfg.tree = r
                trees.append(api.grow_tree(Xd, yd, cfg))
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
            arm[f"T{T}"] = {"ms_per_tree": ms,
                            "root_loss": float(np.mean([t["split_loss"][0] for t in trees])),
                            "train_accuracy": float(np.mean([(api.predict(t, Xd) == y).mean()
                                                             for t in trees])),
                            "nodes": float(np.mean([t["n_nodes"] for t in trees]))}
        res["plain" if n == 0 else f"top{n}_of_{D}"] = arm
    log(f"dft vs plain: {res}")
    return res


def probsearch_vs_pso(api, Xd, yd, K):
    """The swarm (plain and adaptive) against the original SLM's probabilistic
    search (Sec. II-B) at the plain tree's root: split loss and search time
    after T + 1 evaluations of P = 256 candidates."""
    import torch
    res = {}
    for name, prop, apso, Ts in (("pso", 0, False, (10, 50)), ("apso", 0, True, (10, 50)),
                                 ("probabilistic_R16", 2, False, (10, 50, 200, 1000))):
        arm = {}
        for T in Ts:
            cfg = api.TreeConfig(crit=api.ENTROPY, K=K, max_depth=1, min_node=32, P=256, T=T,
                                 bins=256, seed=0, use_graph=True, proposal=prop, ps_R=16,
                                 ps_alpha0=10.0, apso=apso)
            api.grow_tree(Xd, yd, cfg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            losses = []
            for r in range(2):
                cfg.tree = r
                losses.append(api.grow_tree(Xd, yd, cfg)["split_loss"][0])
            torch.cuda.synchronize()
            arm[f"T{T}"] = {"evaluations": T + 1, "root_loss": float(np.mean(losses)),
                            "ms": 1e3 * (time.perf_counter() - t0) / 2}
        res[name] = arm
    log(f"probabilistic search vs pso: {res}")
    return res


def forest_vs_trees(api, Xd, yd, K, n_trees=30):
    """SLM Forest of 30 trees (Sec. V) grown together in one breadth-first
    pass against the same trees grown one per call (same draws)."""
    import torch
    cfg = api.TreeConfig(crit=api.ENTROPY, K=K, max_depth=8, min_node=32, P=256, T=50, bins=256,
                         seed=0, use_graph=True)

    def together():
        cfg.tree = 0
        return api.grow_forest(Xd, yd, cfg, n_trees)

    def one_by_one():
        out = []
        for b in range(n_trees):
            cfg.tree = b
            out.append(api.grow_forest(Xd, yd, cfg, 1))
        return out

    res = {}
    for name, fn in (("together", together), ("one_by_one", one_by_one)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ss = (int(r["sample_splits"][0]) if isinstance(r, dict)
              else sum(int(t["sample_splits"][0]) for t in r))
        res[name] = {"ms": 1e3 * dt, "trees_per_s": n_trees / dt, "sample_splits_per_s": ss / dt,
                     "nodes": int(r["n_nodes"]) if isinstance(r, dict)
                     else sum(int(t["n_nodes"]) for t in r)}
        if name == "together":
            forest = r
        else:
            same = all(np.array_equal(api.forest_tree(forest, b)[k], api.forest_tree(t, 0)[k])
                       for b, t in enumerate(r) for k in ("w", "thr", "left", "right"))
    res["same_trees"] = bool(same)
    res["speedup"] = res["one_by_one"]["ms"] / res["together"]["ms"]
    res["n_trees"] = n_trees
    api._forest_ws.clear()
    log(f"forest vs trees: {res}")
    return res


def boost_rounds(api, Xd, yd, K, rounds=10, lr=0.3):
    """SLR Boost (Friedman's first function, D = 64, N = 1e5) and SLM Boost
    (K-class softmax on the plain-tree data): depth-4 SLR trees, P = 64,
    T = 20, 256 bins; time per round and the training loss."""
    import torch

    from paper_2208_07023_amd import inputs
    N, D = Xd.shape
    Xr, yr = inputs.friedman1(N, D, noise=1.0, seed=1)
    Xrd, yrd = torch.from_numpy(Xr).to(Xd.device), torch.from_numpy(yr).to(Xd.device)
    cfg = api.TreeConfig(crit=api.MSE, K=0, max_depth=4, min_node=32, P=64, T=20, bins=256,
                         seed=0, use_graph=True)
    res = {}
    for name, X, y, nc in (("slr_boost", Xrd, yrd, 0), ("slm_boost", Xd, yd, K)):
        api.boost(X, y, cfg, 1, lr, n_classes=nc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m = api.boost(X, y, cfg, rounds, lr, n_classes=nc)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        F = m["F"]
        if nc:
            loss = float(-torch.log_softmax(F, dim=1)[torch.arange(N, device=F.device),
                                                       y.long()].mean())
            base = float(np.log(nc))
        else:
            loss = float(((y - F[:, 0]) ** 2).mean())
            base = float(((y - y.mean()) ** 2).mean())
        res[name] = {"rounds": rounds, "trees": rounds * max(1, nc), "ms_per_round": 1e3 * dt / rounds,
                     "sample_splits_per_s": int(m["sample_splits"][0]) / dt,
                     "train_loss_start": base, "train_loss_end": loss, "lr": lr}
    log(f"boost: {res}")
    return res


def learned_vs_plain(api, dev, full=False):
    """Learned against random swarm starts at equal node loss.  Pairs are
    harvested from plain-PSO trees (D = 128, K = 5 class mixtures, N
    log-uniform), networks are trained with the library's kernels, and the
    nodes of held-out trees are searched with P = 64 particles from random
    starts and from hybrid starts (M learned seeds, the rest random) until
    each node's global-best loss is within 1 % of a reference search
    (P = 256, T = 200), at most 50 moves.  full=True: the configured scale
    (about 200 k pairs from trees with N in [1e4, 5e5]; a 16-tree bootstrap
    forest on N = 2e6); otherwise a reduced one."""
    from paper_2208_07023_amd import proposal as PL
    D, K, H = 128, 5, 256
    if full:
        n_harvest, n_lo, n_hi, N_eval, n_eval_trees = 2500, 10_000, 500_000, 2_000_000, 16
    else:
        n_harvest, n_lo, n_hi, N_eval, n_eval_trees = 200, 10_000, 100_000, 200_000, 1
    t0 = time.perf_counter()
    S, G, T = PL.harvest(n_harvest, D, K, n_lo, n_hi, seed=7, P=64, T=50, max_depth=8, log=log)
    t_h = time.perf_counter() - t0
    nets, train = {}, {}
    for M in (8, 32, 64):
        t0 = time.perf_counter()
        net, hist = PL.train(S, T, D, K, n_seeds=M, hidden=H, epochs=20, batch=4096)
        train[M] = {"s": time.perf_counter() - t0, "loss_first_last": [hist[0], hist[-1]]}
        nets[M] = net
    res = PL.compare_forest(nets, N_eval, D, K, n_eval_trees, ref_P=256, ref_T=200, P=64,
                            T_max=50, seed=999, log=log)
    out = {"workload": f"harvest {n_harvest} plain-PSO trees (D={D}, K={K}, 4 clusters/class, "
                       f"N log-uniform in [{n_lo}, {n_hi}]); evaluation: {n_eval_trees}-tree "
                       f"bootstrap forest on N={N_eval}; reference P=256, T=200; arms P=64, "
                       "T_max=50, target 1.01 L_ref; hybrid starts: M learned seeds + 64-M random",
           "pairs": int(S.shape[0]), "harvest_s": t_h,
           "train": {str(m): v for m, v in train.items()}, **res}
    log(f"learned vs plain: {out}")
    return out


# ------------------------------------------------------------------ oracle on the host
_ORACLE_JOB = None


def _oracle_init(Xs, y, W, bins, crit, K):
    """Worker set-up: the sample rows, labels and directions, kept per process."""
    global _ORACLE_JOB
    _ORACLE_JOB = (Xs, y, W, bins, crit, K)


def _oracle_chunk(lo_hi):
    """Oracle scans of particles lo .. hi-1 of the job (one BLAS thread):
    FP64 projection, float32 rounding, one histogram scan per particle."""
    from threadpoolctl import threadpool_limits

    from oracle import split as OS
    Xs, y, W, bins, crit, K = _ORACLE_JOB
    lo, hi = lo_hi
    with threadpool_limits(limits=1):
        Z = OS.project(Xs, W[lo:hi]).astype(np.float32)
        for p in range(hi - lo):
            OS.scan_hist(Z[:, p], y, bins, crit, K)
    return hi - lo


def _oracle_rate(Xs, y, W, bins, crit, K, workers, seconds):
    """Oracle sample-splits/s on rows Xs over blocks of the directions W, on
    `workers` processes (1: this process), for about `seconds`."""
    import multiprocessing as mp
    n, P = Xs.shape[0], W.shape[0]
    blk = 4
    blocks = [(lo, min(P, lo + blk)) for lo in range(0, P, blk)]
    done = 0
    if workers == 1:
        _oracle_init(Xs, y, W, bins, crit, K)
        t0 = time.perf_counter()
        i = 0
        while time.perf_counter() - t0 < seconds:
            done += _oracle_chunk(blocks[i % len(blocks)])
            i += 1
        dt = time.perf_counter() - t0
        return done * n / dt, dt, done
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_oracle_init, initargs=(Xs, y, W, bins, crit, K)) as pool:
        pool.map(_oracle_chunk, [(0, 1)] * workers)          # workers started and warm
        t0 = time.perf_counter()
        pending = [pool.apply_async(_oracle_chunk, (blocks[i % len(blocks)],))
                   for i in range(2 * workers)]
        i = 2 * workers
        while pending:
            done += pending.pop(0).get()
            if time.perf_counter() - t0 < seconds:
                pending.append(pool.apply_async(_oracle_chunk, (blocks[i % len(blocks)],)))
                i += 1
        dt = time.perf_counter() - t0
    return done * n / dt, dt, done


def cpu_baseline(screen_data, plain, gpu, seconds=10.0):
    """The FP64 oracle (as it stands) on this host's cores: one root
    evaluation's work (FP64 projection, float32 rounding, one 256-bin
    histogram scan per particle) on a bounded row sample of the headline
    workload, on one core and on all usable cores; the other workloads'
    oracle rates on one core, and their whole-tree CPU times extrapolated
    from the trees' sample-split counts (labelled)."""
    from oracle import screen as OSC
    from oracle import split as OS
    from paper_2208_07023_amd import inputs
    hi = host_info()
    bits, y = screen_data
    n_s = 100_000
    Xs = OSC.bf16_round(inputs.bf16_bits_to_f32(bits[:n_s]))
    Ws = OSC.bf16_round(inputs.random_unit_rows(1024, 256, seed=123).astype(np.float32))
    ys = y[:n_s]
    r1, dt1, p1 = _oracle_rate(Xs, ys, Ws, 256, OS.GINI, 10, 1, seconds)
    rn, dtn, pn = _oracle_rate(Xs, ys, Ws, 256, OS.GINI, 10, hi["usable"], seconds)
    out = {"value": rn, "unit": "sample-splits/s", "cores": hi["usable"], "kind": "oracle",
           "sample": f"{pn} particle scans of {n_s} rows of the screening workload (D=256, "
                     f"bfloat16 data and directions, FP64 projection, 256-bin Gini) on "
                     f"{hi['usable']} worker processes, {dtn:.1f} s",
           "one_core": {"value": r1, "cores": 1,
                        "sample": f"{p1} particle scans of {n_s} rows, {dt1:.1f} s, 1 thread"},
           "host": hi}
    # other workloads: one-core oracle rates on bounded samples
    X2, y2 = plain
    W2 = inputs.random_unit_rows(256, X2.shape[1], seed=123).astype(np.float32)
    r2, _, _ = _oracle_rate(X2[:50_000], y2[:50_000], W2, 256, OS.ENTROPY, 3, 1, seconds / 4)
    X3, y3 = inputs.abs_direction_regression(100_000, 128, seed=0)
    W3 = inputs.random_unit_rows(512, 128, seed=123).astype(np.float32)
    r3, _, _ = _oracle_rate(X3, y3, W3, 256, OS.MSE, 0, 1, seconds / 4)
    est = {}
    for name, rate, key in (("screening_tree", rn, "screening"), ("plain_tree", r2, "plain"),
                            ("regression_tree", r3, "regression")):
        ss = gpu.get(key)
        if ss:
            est[name] = {"oracle_rate_ss_per_s": rate, "sample_splits_per_tree": ss,
                         "extrapolated_cpu_s_per_tree": ss / rate,
                         "cores": hi["usable"] if name == "screening_tree" else 1}
    out["extrapolated"] = est
    # single node (N = 1000, D = 8, P = 32, T = 20, exact scan, Gini): the
    # oracle's whole search timed directly, one thread
    from threadpoolctl import threadpool_limits

    from oracle import pso as OP
    from oracle import tree as OT
    Xc, yc, _ = inputs.two_class_gaussian(1000, 8, seed=0)
    prm = OT.TreeParams(crit=OS.GINI, K=2, P=32, T=20, bins=0)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        OP.run_pso(OT.evaluate_node(Xc.astype(np.float64), yc, prm), 32, 8, 20, 0.7, 1.5, 1.5,
                   0, 0, 0)
        dt = time.perf_counter() - t0
    out["single_node"] = {"ms_per_pso_21_evals": 1e3 * dt, "cores": 1,
                          "sample_splits_per_s": 21 * 1000 * 32 / dt}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain start comparison")
    ap.add_argument("--learned-full", action="store_true",
                    help="run the learned-proposal comparison at its configured scale")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the top-n DFT, probabilistic-search, forest and boosting legs")
    ap.add_argument("--only-headline", action="store_true")
    ap.add_argument("--only-learned", action="store_true",
                    help="only run the learned-vs-plain comparison (with --learned-full at its "
                         "configured scale) and exit")
    ap.add_argument("--root-evals", choices=["screening", "plain", "regression"], default=None,
                    help="only run --reps root evaluations (projection + histogram scan, and "
                         "the re-scoring for the screening tree) of one workload and exit: the "
                         "launches rocprofv3 counter passes read")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--plans", choices=["cached", "rules"], default="cached",
                    help="launch plans of the tree builds: the measured plans cached beside "
                         "the library (default) or the kernels' fitted rules")
    ap.add_argument("--tune-plans", default=None, metavar="PATH",
                    help="only measure the launch plans of the screening, plain and regression "
                         "trees (one tree each) into PATH and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times "
                         "(reference kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(this build runs the split search on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}), flush=True)
        return

    from paper_2208_07023_amd import api
    api.load()
    dev = "cuda"
    if args.tune_plans:
        print(json.dumps(tune_plans(api, args.tune_plans, dev)), flush=True)
        return
    n_plans = api.autotune(0 if args.plans == "rules" else 1)
    log(f"launch plans: {args.plans} ({n_plans} cached)")
    if args.root_evals:
        print(json.dumps(root_evals(api, args.root_evals, args.reps, dev)), flush=True)
        return
    if args.only_learned:
        print(json.dumps(learned_vs_plain(api, dev, full=args.learned_full)), flush=True)
        return
    head, screen_data = headline(api, args, dev)
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "sample-splits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "sample_splits_rescored_per_s": head["sample_splits_rescored_per_s"],
        "kernels": head["kernels"],
        "screening_gpu": head["screening_gpu"],
        "launch_plans": {"kind": args.plans, "cached_plans": n_plans},
    }
    gpu_ss = {"screening": head["config"]["sample_splits_per_tree"]}
    plain = None
    if not args.only_headline:
        p_line, (X2, y2, Xd2, yd2) = plain_tree_line(api, dev)
        out["plain_tree"] = p_line
        plain = (X2, y2)
        gpu_ss["plain"] = int(p_line["sample_splits_per_s"] * p_line["ms_per_tree"] * 1e-3)
        r_line = regression_tree_line(api, dev)
        out["regression_tree"] = r_line
        gpu_ss["regression"] = int(r_line["sample_splits_per_s"] * r_line["ms_per_tree"] * 1e-3)
        out["single_node"] = single_node_line(api, dev)
        if not args.no_extras:
            out["dft_vs_plain"] = dft_vs_plain(api, Xd2, yd2, y2, 3)
            out["probsearch_vs_pso"] = probsearch_vs_pso(api, Xd2, yd2, 3)
            out["forest_vs_trees"] = forest_vs_trees(api, Xd2, yd2, 3)
            out["boost"] = boost_rounds(api, Xd2, yd2, 3)
        if not args.no_learned:
            out["learned_vs_plain"] = learned_vs_plain(api, dev, full=args.learned_full)
    if not args.no_cpu_baseline:
        if plain is None:
            from paper_2208_07023_amd import inputs
            plain = inputs.cluster_mixture(100_000, 64, 3, clusters_per_class=4, mean_std=2.0,
                                           seed=0)
        out["cpu_baseline"] = cpu_baseline(screen_data, plain, gpu_ss)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
