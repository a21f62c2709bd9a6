"""GPU parity of the mixed-precision screening path against the oracle, through
the C ABI: bfloat16 MFMA projection, float32 re-projection of bfloat16 data,
selection of the re-scored particles, merge, swarm step with the global-best
eligibility, and the screened tree.

Bars: integer-valued projections and every index / selection / merge result
bit-exact; Gaussian bfloat16 projections within the forward error bound of a
float32 dot product; trees by held-out accuracy within 0.5 percentage points.
"""
import numpy as np
import pytest
import torch

from oracle import pso as OP
from oracle import screen as SC
from oracle import split as OS
from oracle import tree as OT
from paper_2208_07023_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"
U32 = 2.0 ** -24


def _t(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def _bf16(a):
    """float32 array of bfloat16-representable values -> device bfloat16 tensor."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert np.array_equal(SC.bf16_round(a), a)
    return _t(a).to(torch.bfloat16)


# ------------------------------------------------------------------ projections
@pytest.mark.parametrize("tiled", [False, True, 8, "bf16"])
@pytest.mark.parametrize("D,P,sizes", [
    (8, 32, [1000]),
    (64, 256, [0, 1, 130, 777, 2]),
    (70, 48, [300, 0, 129]),
    (256, 130, [17, 200, 385]),
    (256, 250, [33, 0, 611, 1]),
    (13, 7, [5, 140]),
])
def test_bf16_projection_integer_inputs_bit_exact(gpu_lib, D, P, sizes, tiled):
    api = gpu_lib
    off = inputs.segment_offsets(sizes)
    N, nn = int(off[-1]), len(sizes)
    X = inputs.integer_matrix(N, D, -8, 8, seed=D + P)
    W = inputs.integer_matrix(nn * P, D, -4, 4, seed=D * P + 1)
    Z, zmin, zmax = api.project(_bf16(X), _bf16(W), _t(off), P, tiled=tiled)
    if tiled:
        Z = api.untile_z(Z, P)
    torch.cuda.synchronize()
    Z, zmin, zmax = Z.float().cpu().numpy(), zmin.cpu().numpy(), zmax.cpu().numpy()
    # bfloat16 storage: the exact (integer) projection rounded to nearest even
    store = SC.bf16_round if tiled == "bf16" else (lambda v: v)
    for j in range(nn):
        r0, r1 = off[j], off[j + 1]
        ref = OS.project(X[r0:r1], W[j * P:(j + 1) * P])
        assert np.array_equal(Z[r0:r1], store(ref.astype(np.float32)))
        if r1 > r0:
            assert np.array_equal(zmin[j * P:(j + 1) * P], store(ref.min(0).astype(np.float32)))
            assert np.array_equal(zmax[j * P:(j + 1) * P], store(ref.max(0).astype(np.float32)))
        else:
            assert np.all(np.isposinf(zmin[j * P:(j + 1) * P]))


@pytest.mark.parametrize("D,P,sizes", [(256, 1024, [700, 333]), (128, 96, [513]), (40, 64, [90, 3])])
def test_bf16_projection_gaussian_within_fp32_bound(gpu_lib, D, P, sizes):
    """|Z - X W^T| <= D u sum_d |x_d w_d| + u |Z| with u = 2^-24 (float32
    accumulation of exact bfloat16 products in any order)."""
    api = gpu_lib
    off = inputs.segment_offsets(sizes)
    N, nn = int(off[-1]), len(sizes)
    rng = np.random.default_rng(D + P)
    X = SC.bf16_round(rng.standard_normal((N, D)).astype(np.float32) * 3)
    W = SC.bf16_round(inputs.random_unit_rows(nn * P, D, seed=P).astype(np.float32))
    Z, zmin, zmax = api.project(_bf16(X), _bf16(W), _t(off), P)
    torch.cuda.synchronize()
    Z = Z.cpu().numpy()
    for j in range(nn):
        r0, r1 = off[j], off[j + 1]
        Wj = W[j * P:(j + 1) * P]
        ref = OS.project(X[r0:r1], Wj)
        mag = np.abs(X[r0:r1]).astype(np.float64) @ np.abs(Wj).astype(np.float64).T
        err = np.abs(Z[r0:r1] - ref)
        assert np.all(err <= D * U32 * mag + U32 * np.abs(ref) + 1e-30)
        assert np.array_equal(zmin.cpu().numpy()[j * P:(j + 1) * P], Z[r0:r1].min(0))
        assert np.array_equal(zmax.cpu().numpy()[j * P:(j + 1) * P], Z[r0:r1].max(0))


@pytest.mark.parametrize("D,P,sizes", [(8, 32, [400, 0, 77]), (128, 32, [300, 129]),
                                       (256, 40, [250]), (13, 5, [60, 0, 7]), (100, 33, [70])])
def test_mixed_projection_exact_and_column_alone_identical(gpu_lib, D, P, sizes):
    """bfloat16 X with float32 W: exact on integer-valued inputs, and a column
    recomputed alone (P = 1, the partition) equals the same column among P
    (the re-scoring) bit for bit on Gaussian inputs.  D = 13 and 100 take the
    path for rows that are not whole 16-byte groups."""
    api = gpu_lib
    off = inputs.segment_offsets(sizes)
    N, nn = int(off[-1]), len(sizes)
    Xi = inputs.integer_matrix(N, D, -8, 8, seed=3)
    Wi = inputs.integer_matrix(nn * P, D, -300, 300, seed=4)      # not bfloat16 values
    Z, _, _ = api.project(_bf16(Xi), _t(Wi), _t(off), P, tiled=True)
    Z = api.untile_z(Z, P).cpu().numpy()
    for j in range(nn):
        r0, r1 = off[j], off[j + 1]
        assert np.array_equal(Z[r0:r1], OS.project(Xi[r0:r1], Wi[j * P:(j + 1) * P]).astype(np.float32))
    rng = np.random.default_rng(5)
    X = SC.bf16_round(rng.standard_normal((N, D)).astype(np.float32))
    W = inputs.random_unit_rows(nn * P, D, seed=6).astype(np.float32)
    Zall, _, _ = api.project(_bf16(X), _t(W), _t(off), P, tiled=True)
    Zall = api.untile_z(Zall, P).cpu().numpy()
    for p in (0, P // 2, P - 1):
        W1 = np.ascontiguousarray(W.reshape(nn, P, D)[:, p, :])
        Z1, _, _ = api.project(_bf16(X), _t(W1), _t(off), 1)
        assert np.array_equal(Z1.cpu().numpy()[:, 0], Zall[:, p]), p


@pytest.mark.parametrize("D,P,sizes", [(256, 64, [900, 5]), (100, 33, [70, 0, 41]), (13, 5, [60])])
def test_mixed_projection_gaussian_within_fp32_bound(gpu_lib, D, P, sizes):
    """bfloat16 X with float32 W (the re-scoring; W split into three bfloat16
    parts, every product exact, float32 accumulation): each projection within
    the float32 dot-product bound of the exact value, D u sum |x w| + u |z|,
    widened by 2 % for the three parts' magnitudes (|w1| + |w2| + |w3| <=
    |w| (1 + 2^-7)) and the final addition of the three accumulators."""
    api = gpu_lib
    off = inputs.segment_offsets(sizes)
    N, nn = int(off[-1]), len(sizes)
    rng = np.random.default_rng(D + P)
    X = SC.bf16_round(rng.standard_normal((N, D)).astype(np.float32) * 3)
    W = rng.standard_normal((nn * P, D)).astype(np.float32)
    assert not np.array_equal(SC.bf16_round(W), W)
    Z, _, _ = api.project(_bf16(X), _t(W), _t(off), P, tiled=True)
    Z = api.untile_z(Z, P).cpu().numpy()
    u = 2.0 ** -24
    for j in range(nn):
        r0, r1 = off[j], off[j + 1]
        Wj = W[j * P:(j + 1) * P].astype(np.float64)
        Xj = X[r0:r1].astype(np.float64)
        z64 = Xj @ Wj.T
        bound = 1.02 * (D * u * (np.abs(Xj) @ np.abs(Wj).T) + u * np.abs(z64))
        assert np.all(np.abs(Z[r0:r1].astype(np.float64) - z64) <= bound + 1e-30), j


# ------------------------------------------------------------------ select / gather / merge
@pytest.mark.parametrize("P,k", [(32, 1), (100, 32), (1024, 32), (4096, 64), (7, 7)])
def test_screen_select_matches_oracle(gpu_lib, P, k):
    api = gpu_lib
    nn = 5
    rng = np.random.default_rng(P + k)
    loss = rng.integers(0, 6, nn * P) / 5.0              # many ties
    loss[rng.integers(0, nn * P, nn * P // 8)] = np.inf
    loss[rng.integers(0, nn * P, 4)] = -0.0
    sel = api.screen_select(_t(loss), nn, P, k).cpu().numpy().reshape(nn, k)
    for j in range(nn):
        assert np.array_equal(sel[j], SC.top_k(loss[j * P:(j + 1) * P], k)), j


def test_screen_gather_and_merge(gpu_lib):
    api = gpu_lib
    nn, P, k, D = 3, 50, 8, 19
    rng = np.random.default_rng(2)
    x = rng.standard_normal((nn * P, D))
    sel = np.stack([rng.permutation(P)[:k] for _ in range(nn)]).astype(np.int32)
    W32 = api.screen_gather(_t(x), _t(sel.ravel()), nn, P, k).cpu().numpy()
    assert np.array_equal(W32, x.reshape(nn, P, D)[np.arange(nn)[:, None], sel].reshape(nn * k, D)
                          .astype(np.float32))
    loss = rng.uniform(0, 1, nn * P)
    split = rng.integers(1, 255, nn * P).astype(np.int32)
    thr = rng.standard_normal(nn * P).astype(np.float32)
    lr = rng.uniform(0, 1, nn * k)
    sr = rng.integers(1, 255, nn * k).astype(np.int32)
    tr = rng.standard_normal(nn * k).astype(np.float32)
    L, S_, T_ = _t(loss), _t(split), _t(thr)
    gl = api.screen_merge(_t(sel.ravel()), _t(lr), _t(sr), _t(tr), nn, P, k, L, S_, T_)
    L, S_, T_, gl = (v.cpu().numpy() for v in (L, S_, T_, gl))
    for j in range(nn):
        s = slice(j * P, (j + 1) * P)
        el, es, et = loss[s].copy(), split[s].copy(), thr[s].copy()
        eg = np.full(P, np.inf)
        el[sel[j]] = lr[j * k:(j + 1) * k]
        es[sel[j]] = sr[j * k:(j + 1) * k]
        et[sel[j]] = tr[j * k:(j + 1) * k]
        eg[sel[j]] = lr[j * k:(j + 1) * k]
        assert np.array_equal(L[s], el) and np.array_equal(S_[s], es)
        assert np.array_equal(T_[s], et) and np.array_equal(gl[s], eg)


@pytest.mark.parametrize("crit,K,bins,store", [(OS.GINI, 3, 64, "f32"), (OS.GINI, 3, 64, "bf16"),
                                               (OS.ENTROPY, 4, 256, "bf16"), (OS.MSE, 0, 32, "f32"),
                                               (OS.GINI, 2, 0, "f32")])
def test_screened_evaluation_matches_oracle(gpu_lib, crit, K, bins, store):
    """The whole screened evaluation of several nodes through the C ABI
    (bfloat16 projection, scan, select, gather, float32 re-projection, scan,
    merge) against oracle.screen.  Data X = i/4 and directions x = m/1024
    (10 significant bits: not bfloat16 values, so screen and re-score see
    different projections) keep every partial sum exact in float32, and
    integer targets keep the regression sums exact: losses, splits,
    thresholds, the selection and the global-best eligibility agree bit for
    bit.  store: float32 32-wide tiles, or the bfloat16 8-wide tiles a
    classification histogram search keeps (the exact projections rounded to
    nearest even on both sides)."""
    api = gpu_lib
    sizes = [600, 0, 257, 40] if bins else [300, 2, 41]
    off = inputs.segment_offsets(sizes)
    N, nn, P, k, D = int(off[-1]), len(sizes), 48, 8, 12
    rng = np.random.default_rng(bins + K)
    X = (rng.integers(-16, 17, (N, D)) / 4.0).astype(np.float32)
    x64 = rng.integers(-1023, 1024, (nn * P, D)) / 1024.0
    W32 = x64.astype(np.float32)
    assert not np.array_equal(SC.bf16_round(W32), W32)
    tn = (rng.integers(-5, 6, N).astype(np.float64) if crit == OS.MSE
          else rng.integers(0, K, N).astype(np.int32))
    td = _t(tn)
    offd = _t(off)
    Zs, zmin, zmax = api.project(_bf16(X), _t(SC.bf16_round(W32)).to(torch.bfloat16), offd, P,
                                 tiled="bf16" if store == "bf16" else True)
    scr = api.split_scan(Zs, zmin, zmax, td, K, offd, P, bins, crit)
    sel = api.screen_select(scr["loss"], nn, P, k)
    Wk = api.screen_gather(_t(x64), sel, nn, P, k)
    Zr, rmin, rmax = api.project(_bf16(X), Wk, offd, k, tiled=True)
    res = api.split_scan(Zr, rmin, rmax, td, K, offd, k, bins, crit)
    gl = api.screen_merge(sel, res["loss"], res["split"], res["thr"], nn, P, k,
                          scr["loss"], scr["split"], scr["thr"])
    loss, spl, thr, gl = (v.cpu().numpy() for v in (scr["loss"], scr["split"], scr["thr"], gl))
    for j in range(nn):
        r0, r1 = off[j], off[j + 1]
        s = slice(j * P, (j + 1) * P)
        if r1 - r0 == 0:
            assert np.all(np.isinf(loss[s])) and np.all(np.isinf(gl[s]))
            continue
        ev = SC.evaluate_screened(X[r0:r1], tn[r0:r1], crit, K, bins, k, z_bf16=store == "bf16")
        el, es, et, eg = ev(W32[s])
        assert np.array_equal(spl[s], es) and np.array_equal(thr[s], et)
        if crit == OS.ENTROPY:   # log2 by table and series: within 1e-12 (as every entropy scan)
            assert np.allclose(loss[s], el, rtol=1e-12, atol=0)
            assert np.array_equal(np.isinf(gl[s]), np.isinf(eg))
            fin = np.isfinite(eg)
            assert np.allclose(gl[s][fin], eg[fin], rtol=1e-12, atol=0)
        else:
            assert np.array_equal(loss[s], el) and np.array_equal(gl[s], eg)


def test_pso_step_with_eligibility_bit_exact(gpu_lib):
    api = gpu_lib
    nn, P, D = 4, 64, 10
    st = inputs.random_pso_state(nn, P, D, seed=21, ties=True)
    rng = np.random.default_rng(22)
    gloss = np.full(nn * P, np.inf)
    for j in range(nn):
        pick = rng.permutation(P)[:8]
        gloss[j * P + pick] = st.loss[j * P + pick] + rng.integers(0, 2, 8) / 8.0
    sw = api.pso_alloc(nn, P, D, node_id=np.arange(nn) * 3 + 1)
    for name in ("x", "v", "pbest", "pbest_loss", "gbest", "gbest_loss"):
        getattr(sw, name).copy_(_t(getattr(st, name)))
    sw.gbest_p.copy_(_t(st.gbest_p))
    api.pso_step(sw, _t(st.loss), 0.7, 1.5, 1.5, seed=5, tree=2, it=3, move=True, gloss=_t(gloss))
    ref = OP.pso_step(st.x, st.v, st.pbest, st.pbest_loss, st.gbest, st.gbest_loss, st.gbest_p,
                      st.loss, np.arange(nn) * 3 + 1, nn, P, D, 0.7, 1.5, 1.5, 5, 2, 3, True,
                      gloss=gloss)
    torch.cuda.synchronize()
    for name in ("x", "v", "pbest", "pbest_loss", "gbest", "gbest_loss", "gbest_p"):
        assert np.array_equal(getattr(sw, name).cpu().numpy(), ref[name]), name


# ------------------------------------------------------------------ screened tree
def test_screened_tree_matches_oracle(gpu_lib):
    api = gpu_lib
    Xa, ya = inputs.cluster_mixture(16000, 24, 3, seed=17)
    Xa = SC.bf16_round(Xa)
    X, y, Xt, yt = Xa[:8000], ya[:8000], Xa[8000:], ya[8000:]
    cfg = api.TreeConfig(crit=api.GINI, K=3, max_depth=4, min_node=32, P=64, T=6, bins=64,
                         seed=3, precision=1, rescore_k=8)
    g = api.grow_tree(_bf16(X), _t(y), cfg)
    o = OT.grow_tree(X, y, OT.TreeParams(crit=cfg.crit, K=3, max_depth=4, min_node=32, P=64, T=6,
                                         bins=64, seed=3, precision=1, rescore_k=8))
    Xtd = _t(Xt)
    acc_g = float((api.predict(g, Xtd) == yt).mean())
    acc_o = float((OT.predict(o, Xt) == yt).mean())
    print(f"screened tree held-out accuracy gpu {acc_g:.4f} oracle {acc_o:.4f}; "
          f"nodes {g['n_nodes']} / {len(o.thr)}")
    assert abs(acc_g - acc_o) <= 0.005 + 1e-12
    # same initial swarm: the root's best loss differs only through the
    # rounding order of the screening projection (which particles get re-scored)
    assert g["split_loss"][0] == pytest.approx(o.split_loss[0], rel=1e-2)
    assert g["sample_splits"][0] > 0 and g["sample_splits"][1] * 64 == g["sample_splits"][0] * 8
    # every split's loss is that of the float32 projection the partition used
    n = g["n"]
    for i in range(g["n_nodes"]):
        l, r = g["left"][i], g["right"][i]
        if l >= 0:
            w = (n[l] * g["impurity"][l] + n[r] * g["impurity"][r]) / n[i]
            assert w == pytest.approx(g["split_loss"][i], rel=1e-9, abs=1e-12)


def test_screening_report_against_fp64_oracle(gpu_lib):
    """The screening step's error against the FP64 oracle on a 100 000-row
    sample of the screening workload (D = 256, K = 10, P = 1024, top 32,
    Gini, 256 bins), for two swarms:
    * recall: the oracle's best particle over all 1024 (FP64 projection of
      the bfloat16 data on the FP32 directions, rounded to float32, scanned)
      is among the GPU's screened top 32;
    * gap: the oracle loss of the best re-scored particle against the
      oracle's best, relative;
    * per-particle error: the GPU's screened loss (bfloat16 operands, float32
      accumulation, bfloat16 storage, as in the tree) against the oracle's
      loss of the same particle, relative.
    The numbers are printed; the bars are those the screening must meet to
    serve its purpose (a screened top 32 that holds the best particle)."""
    api = gpu_lib
    N, D, K, P, k, B = 100_000, 256, 10, 1024, 32, 256
    bits, y = inputs.lowrank_mixture(N, D, K, seed=3)
    Xf = inputs.bf16_bits_to_f32(bits)
    Xd = _t(bits.view(np.int16)).view(torch.bfloat16)
    off = _t(np.array([0, N], np.int64))
    yd = _t(y)
    hits, gaps, errs = 0, [], []
    for seed in (11, 12):
        x = OP.init_positions(seed, 0, 0, P, D)           # the oracle's start
        sw = api.pso_alloc(1, P, D, node_id=[0], w_dtype=torch.bfloat16)
        api.pso_init(sw, seed=seed, tree=0)
        # the same Box-Muller start up to the libraries' ulps
        assert np.allclose(sw.x.cpu().numpy(), x, rtol=0, atol=1e-14)
        Zs, zmin, zmax = api.project(Xd, sw.W, off, P, tiled="bf16")
        scr = api.split_scan(Zs, zmin, zmax, yd, K, off, P, B, api.GINI)
        sel = api.screen_select(scr["loss"], 1, P, k).cpu().numpy()
        del Zs
        Z64 = OS.project(Xf, x.astype(np.float32)).astype(np.float32)
        lo = np.array([OS.scan_hist(Z64[:, p], y, B, OS.GINI, K)["loss"] for p in range(P)])
        best = int(np.argmin(lo))
        hits += int(best in set(sel.tolist()))
        gaps.append((lo[sel].min() - lo[best]) / lo[best])
        errs.append(np.abs(scr["loss"].cpu().numpy() - lo) / lo)
    e = np.concatenate(errs)
    print(f"screening vs FP64: recall {hits}/2, gap mean {np.mean(gaps):.2e} max "
          f"{np.max(gaps):.2e}, per-particle error median {np.median(e):.2e} "
          f"p99 {np.quantile(e, 0.99):.2e} max {e.max():.2e}")
    assert hits == 2
    assert max(gaps) <= 1e-3
    assert np.median(e) <= 1e-3 and e.max() <= 1e-2
