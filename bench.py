"""Benchmark: plain SLM tree training on one MI355X, in projected sample-splits/s.

Workload (one step = one tree, the whole split-search path): N = 100 000 rows,
D = 64, 3 classes each a mixture of 4 Gaussian clusters (means ~N(0, 2^2 I),
diagonal variances ~U[0.5, 2]); P = 256 particles, T = 50 moves (51
evaluations) per node, 256-bin histogram scan, entropy criterion, depth 8,
minimum node size 32; all frontier nodes of a depth searched together.
Synthetic seeded data, resident in HBM before the timed region.

Prints one JSON line.  `value` = sum over evaluations of n_node * P divided by
the timed wall time.  `roofline` is the dominant kernel's achieved rate from
HIP-event timings of every launch in one extra (instrumented) tree of the same
workload; `learned_vs_plain` compares learned and random swarm starts at equal
node loss (the second half of the metric); `cpu_baseline` times the FP64
oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "projected sample-splits/s; SLM tree train time, learned vs plain @ equal loss"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and, in a
# second run, WRITE_SIZE (KiB per dispatch, mean over the dispatches of one
# timed and one instrumented tree of this workload), scaled by what the same
# counters read for a plain 1 GiB device copy (FETCH_SIZE 524302 KiB -> x 2.0,
# WRITE_SIZE 1048576 KiB -> x 1.0).  Valid only for the kernel source they were
# taken on (SHA-256 of the file); otherwise the traffic is reported as null.
# Summary and commands: profiles/traffic_plain_tree_N100k_D64_P256.md
TRAFFIC = {
    "k_scan_hist": {"source": "paper_2208_07023_amd/csrc/k_scan.hip",
                    "sha256": "ff9dfdac653262ac9b4ffe12fee175c2807725ac5b8b158f0422af213006f907",
                    "fetch_kib": 43088.5, "write_kib": 4152.8},
    "k_scan_finish_bins": {"source": "paper_2208_07023_amd/csrc/k_scan.hip",
                           "sha256": "ff9dfdac653262ac9b4ffe12fee175c2807725ac5b8b158f0422af213006f907",
                           "fetch_kib": 3174.0, "write_kib": 3096.0},
    "k_project": {"source": "paper_2208_07023_amd/csrc/k_project.hip",
                  "sha256": "e27b8abdd5cb1cd0f31e799308bbb86a24ab450dfe1c5fcaa61baee64f9fe512",
                  "fetch_kib": 10796.4, "write_kib": 83806.5},
}
FETCH_SCALE, WRITE_SCALE = 1048576.0 / 524302.3, 1.0


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the stored counters, or None when
    its source has changed since they were taken."""
    import hashlib
    t = TRAFFIC[kernel]
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
            return None
    return (t["fetch_kib"] * FETCH_SCALE + t["write_kib"] * WRITE_SCALE) * 1024.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(X, y, P, bins, seconds=12.0):
    """Oracle time for root evaluations of the same workload: FP64 projection
    of all N rows on P unit directions, float32 rounding, one histogram scan
    (entropy) per particle.  Single thread (BLAS pinned to one core)."""
    from threadpoolctl import threadpool_limits

    from oracle import split as OS
    from paper_2208_07023_amd import inputs
    W = inputs.random_unit_rows(P, X.shape[1], seed=123).astype(np.float32)
    done, ss, t0 = 0, 0, time.perf_counter()
    with threadpool_limits(limits=1):
        while True:
            Z = OS.project(X, W).astype(np.float32)
            for p in range(P):
                OS.scan_hist(Z[:, p], y, bins, OS.ENTROPY, 3)
                ss += X.shape[0]
                done += 1
                if time.perf_counter() - t0 > seconds:
                    break
            if time.perf_counter() - t0 > seconds:
                break
    dt = time.perf_counter() - t0
    return dict(value=ss / dt, unit="sample-splits/s", cores=1, kind="oracle",
                sample=f"{done} particle scans of a root evaluation (N={X.shape[0]}, D={X.shape[1]}, "
                       f"{bins}-bin entropy) incl. FP64 projection, {dt:.1f} s, 1 thread")


def learned_vs_plain():
    """Learned against random swarm starts at equal node loss: harvest pairs
    from plain-PSO trees (D = 128, K = 5 class mixtures), train the proposal
    network with the library's kernels, then search the nodes of a held-out
    tree (N = 200 000) with P = 64 particles from random and from learned
    starts until each node's global-best loss is within 1% of a reference
    search (P = 256, T = 200), at most 50 moves.  Smaller than the 16-tree,
    N = 2e6 forest of the full evaluation so that the benchmark stays short."""
    from paper_2208_07023_amd import inputs
    from paper_2208_07023_amd import proposal as PL
    D, K, M, H = 128, 5, 64, 256
    t0 = time.perf_counter()
    S, G, T = PL.harvest(100, D, K, 10000, 100000, seed=7, P=64, T=50, max_depth=8)
    t_h = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, hist = PL.train(S, T, D, K, n_seeds=M, hidden=H, epochs=20, batch=1024)
    t_t = time.perf_counter() - t0
    X, y = inputs.cluster_mixture(200_000, D, K, clusters_per_class=4, mean_std=0.8, seed=999)
    res = PL.compare_starts(net, X, y, K, ref_P=256, ref_T=200, P=64, T_max=50)
    r, l = res["random"], res["learned"]
    log(f"learned vs plain: {res}")
    return {"workload": "held-out tree N=200000, D=128, K=5 (4 clusters/class, spread 0.8); "
                        "reference P=256, T=200; arms P=64, T_max=50, target 1.01 L_ref",
            "pairs": int(S.shape[0]), "train_loss_first_last": [hist[0], hist[-1]],
            "harvest_s": t_h, "train_s": t_t,
            "plain": r, "learned": l,
            "speedup_wall": r["ms"] / max(1e-9, l["ms"]),
            "speedup_evals": r["evals"] / max(1, l["evals"])}


def dft_vs_plain(Xd, yd, y, K, reps=3):
    """Swarm in each node's top n DFT channels (Alg. 2) against the swarm in
    all D dimensions, on the benchmark's data: for T = 5, 20, 50 moves, the
    root's split loss, the tree's training accuracy and the time per tree
    (mean of `reps` trees after one warm-up; each depth replayed as a HIP
    graph; the DFT step is inside the timed tree)."""
    import torch

    from paper_2208_07023_amd import api
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


def probsearch_vs_pso(Xd, yd, K):
    """The paper's comparison of the swarm (plain and adaptive, APSO) with the
    original SLM's probabilistic search (Sec. II-B), on the benchmark's data:
    the root's split loss and search time after T + 1 evaluations of P = 256 candidates
    (trees of depth 1; mean of 2 trees after one warm-up; the probabilistic
    search combines the root's 16 best DFT-ranked features, alpha0 = 10)."""
    import torch

    from paper_2208_07023_amd import api
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


def forest_vs_trees(Xd, yd, K, n_trees=30):
    """SLM Forest of n_trees trees (Sec. V: 30 per ensemble) on the benchmark's
    data and tree settings: the forest grown together (one breadth-first pass,
    every depth's nodes of all trees in one swarm loop) against the same trees
    grown one after another (slm_grow_forest with one tree per call and the
    same tree ids, so both arms draw the same bootstrap samples and give the
    same trees).  One warm-up of each arm, then one timed run."""
    import torch

    from paper_2208_07023_amd import api
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
    log(f"forest vs trees: {res}")
    return res


def boost_rounds(Xd, yd, K, rounds=10, lr=0.3):
    """SLR Boost (squared loss, Friedman's first function with D = 64 inputs,
    N = 100000) and SLM Boost (K-class softmax on the benchmark's data): SLR
    trees of depth 4, P = 64, T = 20, 256 bins; time per round and the
    training loss after the last round."""
    import torch

    from paper_2208_07023_amd import api, inputs
    N, D = Xd.shape
    Xr, yr = inputs.friedman1(N, D, noise=1.0, seed=1)
    Xrd, yrd = torch.from_numpy(Xr).cuda(), torch.from_numpy(yr).cuda()
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain start comparison")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-dft", action="store_true",
                    help="skip the top-n DFT channel and probabilistic-search comparisons")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the forest and boosting legs")
    ap.add_argument("--N", type=int, default=100_000)
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

    from paper_2208_07023_amd import api, inputs
    api.load()
    dev = "cuda"
    N, D, K = args.N, 64, 3
    X, y = inputs.cluster_mixture(N, D, K, clusters_per_class=4, mean_std=2.0, seed=0)
    Xd = torch.from_numpy(X).to(dev)
    yd = torch.from_numpy(y).to(dev)
    cfg = api.TreeConfig(crit=api.ENTROPY, K=K, max_depth=8, min_node=32, P=256, T=50, bins=256,
                         seed=0, use_graph=not args.no_graph)
    ws = api.tree_workspace(cfg, N, D, dev)
    torch.cuda.synchronize()

    for w in range(args.warmup):
        cfg.tree = 1000 + w
        api.grow_tree(Xd, yd, cfg, workspace=ws)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    total_ss = 0
    trees = []
    t0 = time.perf_counter()
    host_ms = []
    for k in range(args.steps):
        cfg.tree = k
        t1 = time.perf_counter()
        tr = api.grow_tree(Xd, yd, cfg, workspace=ws)
        host_ms.append(1e3 * (time.perf_counter() - t1))
        total_ss += int(tr["sample_splits"][0])
        trees.append(tr)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} trees in {dt:.3f} s; per tree host ms "
        f"{[round(h, 2) for h in host_ms]}, device ms {[round(t['timing'][0], 2) for t in trees]}")

    # instrumented tree: per-launch HIP events on the launch stream
    cfg.tree = 0
    cfg.profile = True
    cfg.use_graph = False
    prof = api.grow_tree(Xd, yd, cfg, workspace=ws)
    tm = prof["timing"]
    ss_prof = int(prof["sample_splits"][0])
    rows_evals = ss_prof / cfg.P
    scan_bytes = ss_prof * 4 + rows_evals * 4            # Z (4 B/ss) + labels (4 B/row)
    scan_ms = tm[4]
    proj_flops = 2.0 * D * ss_prof
    proj_ms = tm[3]
    scan_gbs = scan_bytes / (scan_ms * 1e-3) / 1e9
    proj_tfs = proj_flops / (proj_ms * 1e-3) / 1e12
    kernels = {
        "scan": {"ms_total": scan_ms, "launches": int(tm[7]), "avg_us": 1e3 * scan_ms / max(1, tm[7]),
                 "GB/s": scan_gbs, "frac_hbm": scan_gbs / HBM_PEAK_GBS},
        "project": {"ms_total": proj_ms, "launches": int(tm[6]), "avg_us": 1e3 * proj_ms / max(1, tm[6]),
                    "TFLOP/s": proj_tfs, "frac_fp32": proj_tfs / FP32_PEAK_TFLOPS},
        "pso_step": {"ms_total": tm[5]},
        "tree_ms_profiled": tm[0],
    }
    # The roofline is the projection's: it is the largest single kernel of the
    # tree (profiles/kernels_plain_tree_N100k_D64_P256.md: 41.6% of GPU time,
    # against 35.4% for the histogram kernel), and its events bracket that one
    # kernel.  The scan step's events bracket two kernels (histogram and
    # multi-chunk finish); it is reported under "kernels" with the traffic of
    # both.
    roof = {"bound": "mfma", "kernel": "k_project_short", "achieved": proj_tfs,
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": proj_tfs / FP32_PEAK_TFLOPS,
            "traffic": measured_traffic("k_project"),
            "flops_per_launch": proj_flops / max(1, tm[6])}
    th, tf = measured_traffic("k_scan_hist"), measured_traffic("k_scan_finish_bins")
    kernels["scan"]["traffic_per_launch"] = th + tf if th is not None and tf is not None else None
    kernels["scan"]["bytes_per_launch"] = scan_bytes / max(1, tm[7])

    acc = float((api.predict(trees[0], Xd) == y).mean())
    out = {
        "metric": METRIC,
        "value": total_ss / dt,
        "unit": "sample-splits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain SLM tree: N={N}, D={D}, K={K} (4 Gaussian clusters/class), "
                               f"P=256, T=50, 256-bin histogram, entropy, depth 8, min node 32",
                   "nodes_per_tree": int(trees[0]["n_nodes"]),
                   "sample_splits_per_tree": total_ss // args.steps,
                   "train_accuracy": acc,
                   "hip_graph": cfg.use_graph or not args.no_graph},
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_dft:
        out["dft_vs_plain"] = dft_vs_plain(Xd, yd, y, K)
        out["probsearch_vs_pso"] = probsearch_vs_pso(Xd, yd, K)
    if not args.no_ensemble:
        out["forest_vs_trees"] = forest_vs_trees(Xd, yd, K)
        out["boost"] = boost_rounds(Xd, yd, K)
    if not args.no_learned:
        out["learned_vs_plain"] = learned_vs_plain()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, y, cfg.P, cfg.bins)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
