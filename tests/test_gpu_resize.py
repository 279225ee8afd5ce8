"""Parity of the scale-to-common-size mode (bilinear resize, Section 4.1)
with the FP64 oracle, through cfsim_score and cfsim_score_batch."""
import numpy as np
import pytest

import oracle
from cfgsynth import CFG, Grammar, config_graphs, make_cfg
from tests.parity import base_status, check_margin, check_matching, check_S, oracle_pair, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02423_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(cf):
    return cf.Context(0)


def _graphs(sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        if n == 1:
            out.append(CFG(1, np.array([0], np.int32), np.array([0], np.int32), np.array([3.0])))
        else:
            out.append(make_cfg(n, Grammar(counts="trip"), rng))
    return out


def _check(S, match, res, ref, dtype):
    assert S.shape == ref.S.shape
    er = check_S(S, ref.S, dtype)
    if dtype == "f64":
        assert res["iters"] == ref.iters and base_status(res["status"]) == ref.status
        assert abs(res["nu"] - ref.nu) <= 1e-10 * max(ref.nu, 1.0)
    check_margin(res["margin"], S, match, dtype)
    check_matching(S, match, ref.S, dtype, er)
    S64 = S.astype(np.float64)
    assert abs(res["score"] - sum(S64[i, j] for i, j in enumerate(match) if j >= 0)) < 1e-12


@pytest.mark.parametrize("nA,nB", [(9, 30), (30, 9), (12, 16), (16, 16), (1, 5), (5, 1), (70, 45), (3, 128),
                                   (127, 128)])
def test_resize_plain_fp64(cf, ctx, nA, nB):
    graphs = _graphs([nA, nB], seed=nA * 131 + nB)
    gs = cf.pack(ctx, graphs)
    r = cf.score(ctx, gs, 0, 1, dtype="f64", resize="bilinear")
    ref = oracle_pair(graphs, 0, 1, resize="bilinear")
    _check(r["S"], r["match"], r, ref, "f64")


def test_resize_workload0_pair(cf, ctx):
    w = config_graphs(0)
    gs = cf.pack(ctx, w["graphs"])
    r = cf.score(ctx, gs, 0, 1, dtype="f64", resize="bilinear")
    ref = oracle_pair(w["graphs"], 0, 1, resize="bilinear")
    assert r["S"].shape == (16, 16)
    _check(r["S"], r["match"], r, ref, "f64")


@pytest.mark.parametrize("max_iter,tol", [(1, 1e-12), (2, 1e-12), (3, 0.0), (8, 0.0), (200, 1e-4)])
def test_resize_iteration_controls(cf, ctx, max_iter, tol):
    graphs = _graphs([20, 37], seed=17)
    gs = cf.pack(ctx, graphs)
    r = cf.score(ctx, gs, 1, 0, dtype="f64", max_iter=max_iter, tol=tol, resize="bilinear")
    ref = oracle_pair(graphs, 1, 0, max_iter, tol, resize="bilinear")
    _check(r["S"], r["match"], r, ref, "f64")


def test_resize_degenerate_pair(cf, ctx):
    graphs = _graphs([12], seed=2)
    graphs.append(CFG(5, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([0.0, 0.0])))
    gs = cf.pack(ctx, graphs)
    r = cf.score(ctx, gs, 1, 0, dtype="f64", resize="bilinear")
    ref = oracle_pair(graphs, 1, 0, resize="bilinear")
    assert ref.status == oracle.DEGENERATE and base_status(r["status"]) == cf.DEGENERATE
    _check(r["S"], r["match"], r, ref, "f64")


def test_resize_batch_fp32_workload1_subset(cf, ctx):
    w = config_graphs(1, scale=10 / 256)
    g = w["graphs"]
    gs = cf.pack(ctx, g)
    res, matches, Ss = cf.score_batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", resize="bilinear",
                                      want_S=True)
    assert len(res) == 45
    for p in range(len(res)):
        ref = oracle_pair(g, int(w["pair_a"][p]), int(w["pair_b"][p]), resize="bilinear")
        assert Ss[p].shape == ref.S.shape
        er = check_S(Ss[p], ref.S, "f32")
        check_margin(res["margin"][p], Ss[p], matches[p], "f32")
        check_matching(Ss[p], matches[p], ref.S, "f32", er)


def test_resize_batch_fp64_agrees_with_plain_and_replays(cf, ctx):
    graphs = _graphs([6, 20, 33, 64, 90], seed=8)
    pa, pb = np.triu_indices(len(graphs), k=0)
    pa, pb = pa.astype(np.int32), pb.astype(np.int32)
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, pa, pb, dtype="f64", resize="bilinear", want_S=True)
    b.run()
    torch.cuda.synchronize()
    r1, S1 = b.results().tobytes(), b.S.clone()
    Ss, ms, res = b.S_list(), b.matches(), b.results()
    for p in range(len(pa)):
        ref = oracle_pair(graphs, int(pa[p]), int(pb[p]), resize="bilinear")
        assert res["iters"][p] == ref.iters and base_status(res["status"][p]) == ref.status
        er = check_S(Ss[p], ref.S, "f64")
        check_margin(res["margin"][p], Ss[p], ms[p], "f64")
        check_matching(Ss[p], ms[p], ref.S, "f64", er)
    for _ in range(2):
        b.res.zero_()
        b.run()
        torch.cuda.synchronize()
        assert b.results().tobytes() == r1 and torch.equal(b.S, S1)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_resized_batch_routes_lds_global_and_tiled_pairs(cf, ctx, dtype):
    """One call with pairs the LDS kernels hold in their resized mode (M x m
    state, M x M matching), pairs beyond LDS for the global-memory kernel
    (state and S in a workspace slot) and pairs for the tiled path (smaller
    graph over 128 nodes), against the oracle; equal sizes, a one-node graph
    and a degenerate graph included."""
    sizes = [128, 120, 9, 64, 37, 100, 1, 5, 77, 200, 150]
    graphs = _graphs(sizes, seed=33)
    graphs.append(CFG(6, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([0.0, 0.0])))
    pa = np.array([0, 9, 0, 2, 3, 4, 5, 6, 7, 8, 11, 3, 4, 8], np.int32)
    pb = np.array([1, 10, 2, 3, 4, 5, 1, 7, 3, 0, 2, 3, 8, 4], np.int32)
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, pa, pb, dtype=dtype, resize="bilinear", want_S=True)
    buckets = b.buckets()
    assert buckets[0] == cf.NUM_BUCKETS - 2          # 128 x 120: the global-memory kernel
    assert buckets[1] == cf.NUM_BUCKETS - 1          # 200 x 150: the tiled path
    lds = buckets < cf.NUM_BUCKETS - 2
    if dtype == "f32":
        assert lds[2:].all()                         # the rest on the LDS kernels
    else:                                            # FP64: M x M matching beyond ~99 nodes is not in LDS
        assert lds.sum() >= 8
    b.run()
    torch.cuda.synchronize()
    res, ms, Ss = b.results(), b.matches(), b.S_list()
    for p in range(len(pa)):
        ref = oracle_pair(graphs, int(pa[p]), int(pb[p]), resize="bilinear")
        assert Ss[p].shape == ref.S.shape
        if dtype == "f64":
            assert res["iters"][p] == ref.iters and base_status(res["status"][p]) == ref.status, p
        er = check_S(Ss[p], ref.S, dtype)
        check_margin(res["margin"][p], Ss[p], ms[p], dtype)
        check_matching(Ss[p], ms[p], ref.S, dtype, er)


@pytest.mark.parametrize("max_iter,tol", [(1, 1e-12), (2, 1e-12), (3, 0.0), (8, 0.0), (200, 1e-4)])
def test_resized_batch_iteration_controls(cf, ctx, max_iter, tol):
    graphs = _graphs([20, 37, 64, 9], seed=17)
    pa = np.array([1, 2, 3], np.int32)
    pb = np.array([0, 1, 2], np.int32)
    gs = cf.pack(ctx, graphs)
    res, ms, Ss = cf.score_batch(ctx, gs, pa, pb, dtype="f64", max_iter=max_iter, tol=tol, resize="bilinear",
                                 want_S=True)
    for p in range(len(pa)):
        ref = oracle_pair(graphs, int(pa[p]), int(pb[p]), max_iter, tol, resize="bilinear")
        _check(Ss[p], ms[p], res[p], ref, "f64")
