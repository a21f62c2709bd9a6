"""GPU parity of the HIP kernels against the FP64 oracle, through the C ABI.

Bars: integer/index results (counts, chosen splits, thresholds, RNG draws,
swarm updates) bit-exact; FP32 projections within the forward error bound of
an FP32 dot product; losses within 1e-5 relative (in practice far tighter,
stated per test).
"""
import numpy as np
import pytest
import torch

from oracle import pso as OP
from oracle import screen as SC
from oracle import split as OS
from paper_2208_07023_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


# ------------------------------------------------------------------ projection
@pytest.mark.parametrize("tiled", [False, True, 8])
@pytest.mark.parametrize("D,P,sizes", [
    (8, 32, [1000]),
    (16, 20, [45, 64, 0, 3]),
    (40, 48, [100, 33, 0, 70]),
    (64, 256, [0, 1, 130, 777, 2]),
    (70, 48, [300, 0, 129]),
    (130, 1, [257, 64]),
    (256, 130, [17, 200]),
])
def test_project_integer_inputs_bit_exact(gpu_lib, D, P, sizes, tiled):
    api = gpu_lib
    off = inputs.segment_offsets(sizes)
    N, nn = int(off[-1]), len(sizes)
    X = inputs.integer_matrix(N, D, -8, 8, seed=D + P)
    W = inputs.integer_matrix(nn * P, D, -4, 4, seed=D * P + 1)
    Z, zmin, zmax = api.project(_t(X), _t(W), _t(off), P, tiled=tiled)
    if tiled:
        w = 32 if tiled is True else tiled
        assert Z.shape == ((P + w - 1) // w, N, w)
        Z = api.untile_z(Z, P)
    torch.cuda.synchronize()
    Z, zmin, zmax = Z.cpu().numpy(), zmin.cpu().numpy(), zmax.cpu().numpy()
    for j in range(nn):
        r0, r1 = off[j], off[j + 1]
        ref = OS.project(X[r0:r1], W[j * P:(j + 1) * P])
        assert np.array_equal(Z[r0:r1], ref.astype(np.float32))
        if r1 > r0:
            assert np.array_equal(zmin[j * P:(j + 1) * P], ref.min(0).astype(np.float32))
            assert np.array_equal(zmax[j * P:(j + 1) * P], ref.max(0).astype(np.float32))
        else:
            assert np.all(np.isposinf(zmin[j * P:(j + 1) * P]))
            assert np.all(np.isneginf(zmax[j * P:(j + 1) * P]))


@pytest.mark.parametrize("D,P", [(8, 32), (64, 256), (128, 64), (200, 33)])
def test_project_gaussian_within_fp32_bound(gpu_lib, D, P):
    api = gpu_lib
    sizes = [513, 1, 1200]
    off = inputs.segment_offsets(sizes)
    rng = np.random.default_rng(D)
    X = rng.standard_normal((int(off[-1]), D)).astype(np.float32)
    W = inputs.random_unit_rows(len(sizes) * P, D, seed=P).astype(np.float32)
    Z, _, _ = api.project(_t(X), _t(W), _t(off), P)
    Z = Z.cpu().numpy().astype(np.float64)
    u = 2.0 ** -24
    gam = D * u / (1 - D * u)
    for j in range(len(sizes)):
        r0, r1 = off[j], off[j + 1]
        Wj = W[j * P:(j + 1) * P]
        ref = OS.project(X[r0:r1], Wj)
        mag = np.abs(X[r0:r1].astype(np.float64)) @ np.abs(Wj.astype(np.float64)).T
        assert np.all(np.abs(Z[r0:r1] - ref) <= gam * mag + 1e-30)


def test_project_column_recomputed_alone_is_bit_identical(gpu_lib):
    """The partition recomputes the winning particle's column with P = 1; it
    must reproduce the bits the scan binned."""
    api = gpu_lib
    sizes = [3000, 1777]
    off = inputs.segment_offsets(sizes)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((int(off[-1]), 64)).astype(np.float32)
    P = 256
    W = inputs.random_unit_rows(2 * P, 64, seed=2).astype(np.float32)
    Z, _, _ = api.project(_t(X), _t(W), _t(off), P)
    for p in (0, 31, 32, 200, 255):
        W1 = np.stack([W[p], W[P + p]])
        Z1, _, _ = api.project(_t(X), _t(W1), _t(off), 1)
        assert torch.equal(Z1[:, 0], Z[:, p])


# ------------------------------------------------------------------ histogram scan
def _scan_case(api, sizes, P, B, crit, K, kind, seed, tiled=False):
    off = inputs.segment_offsets(sizes)
    N = int(off[-1])
    Z = inputs.projected_features(N, P, seed=seed, kind=kind)
    if tiled == "bf16":   # bfloat16 storage: the scan reads these values exactly
        Z = SC.bf16_round(Z)
    rng = np.random.default_rng(seed + 1)
    if crit == OS.MSE:
        tgt = rng.normal(2.0, 1.5, size=N)
        tt = torch.float64
    else:
        tgt = rng.integers(0, K, size=N).astype(np.int32)
        tt = torch.int32
    # zmin / zmax are inputs of the scan (the projection writes them)
    zmin = np.full(len(sizes) * P, np.inf, np.float32)
    zmax = np.full(len(sizes) * P, -np.inf, np.float32)
    for j in range(len(sizes)):
        if sizes[j]:
            zmin[j * P:(j + 1) * P] = Z[off[j]:off[j + 1]].min(0)
            zmax[j * P:(j + 1) * P] = Z[off[j]:off[j + 1]].max(0)
    if tiled == "bf16":
        Zd = api.tile_z(_t(Z), P, 8).to(torch.bfloat16)
    else:
        Zd = api.tile_z(_t(Z), P, 32 if tiled is True else tiled) if tiled else _t(Z)
    out = api.split_scan(Zd, _t(zmin), _t(zmax), _t(tgt, tt), K if crit != OS.MSE else 0,
                         _t(off), P, B, crit, hist=True, sums=crit == OS.MSE)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    ref = OS.split_scan(Z, tgt, off, P, B, crit, K)
    return got, ref


@pytest.mark.parametrize("tiled", [False, True, 8, "bf16"])
@pytest.mark.parametrize("crit", [OS.GINI, OS.ENTROPY])
@pytest.mark.parametrize("B,K,P,kind", [
    (256, 3, 32, "gauss"), (256, 2, 8, "dups"), (16, 10, 20, "gauss"), (2, 3, 5, "gauss"),
    (3, 4, 64, "dups"), (256, 3, 40, "const"), (100, 16, 3, "gauss"),
])
def test_hist_scan_classification_exact(gpu_lib, crit, B, K, P, kind, tiled):
    # nodes: empty, single row, small, one spanning several 2048-row chunks, ragged tail
    sizes = [0, 1, 37, 5000, 301]
    got, ref = _scan_case(gpu_lib, sizes, P, B, crit, K, kind, seed=B * 7 + K, tiled=tiled)
    assert np.array_equal(got["counts"].astype(np.int64), ref["counts"])
    assert np.array_equal(got["split"], ref["split"])
    assert np.array_equal(got["thr"], ref["thr"])
    fin = np.isfinite(ref["loss"])
    assert np.array_equal(np.isfinite(got["loss"]), fin)
    if crit == OS.GINI:
        assert np.array_equal(got["loss"][fin], ref["loss"][fin])          # bit-exact Gini
    else:
        assert np.allclose(got["loss"][fin], ref["loss"][fin], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("crit", [OS.GINI, OS.ENTROPY])
@pytest.mark.parametrize("B,K,P,kind,tiled", [
    (256, 3, 32, "gauss", True), (16, 10, 20, "gauss", False), (3, 4, 64, "dups", True),
    (100, 16, 3, "gauss", True), (256, 2, 40, "const", False), (256, 10, 44, "gauss", 8),
    (64, 3, 17, "dups", 8), (256, 10, 44, "gauss", "bf16"), (200, 3, 37, "dups", "bf16"),
])
def test_hist_scan_classification_large_node(gpu_lib, crit, B, K, P, kind, tiled):
    # a node of many chunks among few nodes: finished one bin per thread
    sizes = [45000, 7]
    got, ref = _scan_case(gpu_lib, sizes, P, B, crit, K, kind, seed=B + K + P, tiled=tiled)
    assert np.array_equal(got["counts"].astype(np.int64), ref["counts"])
    assert np.array_equal(got["split"], ref["split"])
    assert np.array_equal(got["thr"], ref["thr"])
    fin = np.isfinite(ref["loss"])
    assert np.array_equal(np.isfinite(got["loss"]), fin)
    if crit == OS.GINI:
        assert np.array_equal(got["loss"][fin], ref["loss"][fin])
    else:
        assert np.allclose(got["loss"][fin], ref["loss"][fin], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("tiled", [False, True, 8])
@pytest.mark.parametrize("B,P,kind", [(256, 16, "gauss"), (64, 33, "dups"), (7, 4, "gauss")])
def test_hist_scan_regression(gpu_lib, B, P, kind, tiled):
    sizes = [0, 2, 45, 4500, 600]
    got, ref = _scan_case(gpu_lib, sizes, P, B, OS.MSE, 0, kind, seed=B + P, tiled=tiled)
    assert np.array_equal(got["counts"].astype(np.int64), ref["counts"])
    # per-bin FP64 sums: atomics in any order, error ~ n * u * sum|y|
    assert np.allclose(got["sums"], ref["sums"], rtol=1e-12, atol=1e-9)
    fin = np.isfinite(ref["loss"])
    assert np.array_equal(np.isfinite(got["loss"]), fin)
    assert np.allclose(got["loss"][fin], ref["loss"][fin], rtol=1e-9, atol=1e-12)
    mism = np.nonzero(got["split"] != ref["split"])[0]
    # a different split only where the oracle's best and the GPU's pick are a near-tie
    for i in mism:
        assert abs(got["loss"][i] - ref["loss"][i]) <= 1e-9 * abs(ref["loss"][i])


def _assert_scan_matches(got, ref, crit):
    assert np.array_equal(got["counts"].astype(np.int64), ref["counts"])
    fin = np.isfinite(ref["loss"])
    assert np.array_equal(np.isfinite(got["loss"]), fin)
    if crit == OS.MSE:
        assert np.allclose(got["sums"], ref["sums"], rtol=1e-12, atol=1e-9)
        assert np.allclose(got["loss"][fin], ref["loss"][fin], rtol=1e-9, atol=1e-12)
        for i in np.nonzero(got["split"] != ref["split"])[0]:
            assert abs(got["loss"][i] - ref["loss"][i]) <= 1e-9 * abs(ref["loss"][i])
        return
    assert np.array_equal(got["split"], ref["split"])
    assert np.array_equal(got["thr"], ref["thr"])
    if crit == OS.GINI:
        assert np.array_equal(got["loss"][fin], ref["loss"][fin])
    else:
        assert np.allclose(got["loss"][fin], ref["loss"][fin], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("w,crit,K", [(8, OS.GINI, 3), (8, OS.ENTROPY, 10), (8, OS.MSE, 0),
                                      (32, OS.GINI, 3), (32, OS.ENTROPY, 10), (32, OS.MSE, 0),
                                      ("bf16", OS.GINI, 3), ("bf16", OS.ENTROPY, 10)])
def test_hist_scan_every_tile_width(gpu_lib, tmp_path, w, crit, K):
    """Every work-group particle tile (4, 8, 16, 32; plans forced through the
    plan cache) reads Z in the 8- and 32-particle layouts and the 8-particle
    bfloat16 one: P = 44 leaves a ragged last tile, the 5000-row node spans
    five 1024-row chunks."""
    import json
    api = gpu_lib
    sizes = [0, 1, 37, 5000, 301]
    P, B = 44, 256
    N = sum(sizes)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    kk = 1 if crit == OS.MSE else K
    key = f"scan/{arch}/N{N}/n8/P{P}/B{B}/K{kk}/c{crit}"
    kt = 5 if crit == OS.MSE else (K if K <= 4 else (8 if K <= 8 else 16))
    for pt in (4, 8, 16, 32):
        if pt * kt > 128:
            continue
        path = tmp_path / f"plans_{pt}.json"
        path.write_text(json.dumps({"plans": {key: [pt, 1024]}}))
        try:
            assert api.autotune(1, str(path)) == 1
            got, ref = _scan_case(api, sizes, P, B, crit, K, "gauss", seed=pt + len(str(w)),
                                  tiled=w)
        finally:
            api.autotune(1)
        _assert_scan_matches(got, ref, crit)


def test_hist_scan_beyond_256_full_chunks(gpu_lib):
    """More rows than 256 chunks of the counter limit (65472 rows) hold: the
    plan's chunks stop at the limit and the accumulator takes more slots
    (a 17 000 000-row node and a small one; P = 4, K = 2, Gini, 64 bins)."""
    sizes = [17_000_000, 5]
    got, ref = _scan_case(gpu_lib, sizes, 4, 64, OS.GINI, 2, "gauss", seed=31)
    _assert_scan_matches(got, ref, OS.GINI)


@pytest.mark.parametrize("sizes", [[9000, 3000], [40000]])
def test_hist_scan_reuses_zeroed_workspace(gpu_lib, sizes):
    """Two calls in a row on the same workspace (multi-chunk nodes, both
    finish kernels) agree."""
    a, ref = _scan_case(gpu_lib, sizes, 32, 256, OS.GINI, 3, "gauss", seed=5)
    b, _ = _scan_case(gpu_lib, sizes, 32, 256, OS.GINI, 3, "gauss", seed=5)
    for k in ("counts", "split", "loss", "thr"):
        assert np.array_equal(a[k], b[k])
    assert np.array_equal(a["split"], ref["split"])


# ------------------------------------------------------------------ exact scan
@pytest.mark.parametrize("crit,K", [(OS.GINI, 2), (OS.ENTROPY, 5), (OS.MSE, 0)])
@pytest.mark.parametrize("kind,P,tiled", [("gauss", 32, False), ("dups", 32, False),
                                          ("gauss", 40, True), ("dups", 21, 8)])
def test_exact_scan(gpu_lib, crit, K, kind, P, tiled):
    sizes = [1000, 0, 1, 2, 333]
    got, ref = _scan_case(gpu_lib, sizes, P, 0, crit, K, kind, seed=17 + crit, tiled=tiled)
    fin = np.isfinite(ref["loss"])
    assert np.array_equal(np.isfinite(got["loss"]), fin)
    if crit == OS.MSE:
        assert np.allclose(got["loss"][fin], ref["loss"][fin], rtol=1e-9, atol=1e-12)
        for i in np.nonzero(got["split"] != ref["split"])[0]:
            assert abs(got["loss"][i] - ref["loss"][i]) <= 1e-9 * abs(ref["loss"][i])
    else:
        assert np.array_equal(got["split"], ref["split"])
        assert np.array_equal(got["thr"], ref["thr"])
        if crit == OS.GINI:
            assert np.array_equal(got["loss"][fin], ref["loss"][fin])
        else:
            assert np.allclose(got["loss"][fin], ref["loss"][fin], rtol=1e-12)


# ------------------------------------------------------------------ swarm
def test_pso_init_matches_oracle(gpu_lib):
    api = gpu_lib
    nodes = [0, 5, 12]
    P, D = 40, 9
    sw = api.pso_alloc(3, P, D, nodes)
    api.pso_init(sw, seed=123, tree=2)
    x = sw.x.cpu().numpy()
    for j, nid in enumerate(nodes):
        ref = OP.init_positions(123, 2, nid, P, D)
        # device libm (log, cos, sin) vs host: a few ulps
        assert np.allclose(x[j * P:(j + 1) * P], ref, rtol=0, atol=4e-15)
    W = sw.W.cpu().numpy()
    assert np.mean(W == x.astype(np.float32)) == 1.0
    assert torch.equal(sw.pbest, sw.x) and torch.all(sw.v == 0)
    assert torch.all(torch.isinf(sw.pbest_loss)) and torch.all(sw.gbest_p == -1)
    assert torch.equal(sw.gbest, sw.x.view(3, P, D)[:, 0])


@pytest.mark.parametrize("ties", [False, True])
@pytest.mark.parametrize("P,D", [(32, 8), (300, 17), (1024, 256)])
def test_pso_step_bit_exact(gpu_lib, ties, P, D):
    api = gpu_lib
    nn = 3
    st = inputs.random_pso_state(nn, P, D, seed=P + D, ties=ties)
    node_id = np.array([1, 4, 9], dtype=np.int32)
    sw = api.pso_alloc(nn, P, D, node_id)
    for name in ("x", "v", "pbest", "pbest_loss", "gbest", "gbest_loss"):
        getattr(sw, name).copy_(_t(getattr(st, name)).view_as(getattr(sw, name)))
    sw.gbest_p.copy_(_t(st.gbest_p))
    loss = _t(st.loss)
    api.pso_step(sw, loss, 0.7, 1.5, 1.5, seed=77, tree=3, it=5, move=True)
    ref = OP.pso_step(st.x, st.v, st.pbest, st.pbest_loss, st.gbest, st.gbest_loss, st.gbest_p,
                      st.loss, node_id, nn, P, D, 0.7, 1.5, 1.5, 77, 3, 5, True)
    torch.cuda.synchronize()
    for name in ("x", "v", "pbest", "pbest_loss", "gbest", "gbest_loss"):
        assert np.array_equal(getattr(sw, name).cpu().numpy().reshape(ref[name].shape), ref[name]), name
    improved = ref["gbest_loss"] < st.gbest_loss
    gp = sw.gbest_p.cpu().numpy()
    assert np.array_equal(gp[improved], ref["gbest_p"][improved])
    assert np.array_equal(sw.W.cpu().numpy(), ref["x"].astype(np.float32))


def test_pso_step_without_move_only_updates_bests(gpu_lib):
    api = gpu_lib
    st = inputs.random_pso_state(2, 16, 4, seed=3)
    sw = api.pso_alloc(2, 16, 4, [0, 1])
    for name in ("x", "v", "pbest", "pbest_loss", "gbest", "gbest_loss"):
        getattr(sw, name).copy_(_t(getattr(st, name)).view_as(getattr(sw, name)))
    x0 = sw.x.clone()
    api.pso_step(sw, _t(st.loss), 0.7, 1.5, 1.5, 1, 0, 1, move=False)
    assert torch.equal(sw.x, x0)
    ref = OP.pso_step(st.x, st.v, st.pbest, st.pbest_loss, st.gbest, st.gbest_loss, st.gbest_p,
                      st.loss, np.array([0, 1]), 2, 16, 4, 0.7, 1.5, 1.5, 1, 0, 1, False)
    assert np.array_equal(sw.pbest_loss.cpu().numpy(), ref["pbest_loss"])
    assert np.array_equal(sw.gbest.cpu().numpy(), ref["gbest"])
