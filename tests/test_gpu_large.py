"""Parity of the large-pair path (cfsim_score_large) with the FP64 oracle."""
import os

import numpy as np
import pytest

import oracle
from cfgsynth import CFG, Grammar, config_graphs, make_cfg
from tests.parity import base_status, check_margin, check_matching, check_S, oracle_pair, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "workload2_oracle.npz")


@pytest.fixture(scope="module")
def cf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02423_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(cf):
    return cf.Context(0)


def _large(cf, ctx, graphs, pa, pb, dtype, max_iter=200, tol=1e-12, want_S=True):
    gs = cf.pack(ctx, graphs)
    return cf.score_batch(ctx, gs, np.asarray(pa, np.int32), np.asarray(pb, np.int32), dtype=dtype,
                          max_iter=max_iter, tol=tol, want_S=want_S, path="large")


def _sizes_graphs(sizes, seed):
    rng = np.random.default_rng(seed)
    g = Grammar(w_seq=0.70, w_ifthen=0.08, w_ifelse=0.07, w_loop=0.15, p_selfloop=0.05, max_loop_depth=4,
                counts="trip")
    return [make_cfg(n, g, rng) for n in sizes]


@pytest.mark.parametrize("nA,nB", [(5, 9), (70, 45), (64, 32), (65, 33), (130, 97), (257, 300)])
def test_large_fp64_ragged_tiles(cf, ctx, nA, nB):
    graphs = _sizes_graphs([nA, nB], seed=nA * 1000 + nB)
    res, matches, Ss = _large(cf, ctx, graphs, [0], [1], "f64")
    ref = oracle_pair(graphs, 0, 1)
    assert Ss[0].shape == ref.S.shape
    er = check_S(Ss[0], ref.S, "f64")
    assert res["iters"][0] == ref.iters and base_status(res["status"][0]) == ref.status
    assert abs(res["nu"][0] - ref.nu) <= 1e-10 * ref.nu
    check_margin(res["margin"][0], Ss[0], matches[0], "f64")
    check_matching(Ss[0], matches[0], ref.S, "f64", er)
    S64 = Ss[0].astype(np.float64)
    assert abs(res["score"][0] - sum(S64[i, j] for i, j in enumerate(matches[0]) if j >= 0)) < 1e-12


@pytest.mark.parametrize("max_iter,tol", [(1, 1e-12), (2, 1e-12), (3, 0.0), (4, 0.0), (7, 1e-12), (200, 1e-3)])
def test_large_iteration_controls(cf, ctx, max_iter, tol):
    graphs = _sizes_graphs([90, 70], seed=5)
    res, matches, Ss = _large(cf, ctx, graphs, [0], [1], "f64", max_iter=max_iter, tol=tol)
    ref = oracle_pair(graphs, 0, 1, max_iter, tol)
    assert res["iters"][0] == ref.iters and base_status(res["status"][0]) == ref.status
    er = check_S(Ss[0], ref.S, "f64")
    if np.isfinite(ref.delta):
        assert abs(res["delta"][0] - ref.delta) <= 1e-9 * max(ref.delta, 1e-300) + 1e-15
    else:
        assert np.isinf(res["delta"][0])
    check_margin(res["margin"][0], Ss[0], matches[0], "f64")
    check_matching(Ss[0], matches[0], ref.S, "f64", er)


def test_large_converging_pair(cf, ctx):
    # a path against a self-loop pair: the coupled iteration settles fast
    graphs = [CFG(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1.0, 1.0])),
              CFG(2, np.array([0, 0, 1], np.int32), np.array([0, 1, 1], np.int32), np.array([1.0, 2.0, 1.0]))]
    res, matches, Ss = _large(cf, ctx, graphs, [0, 1], [1, 0], "f64")
    for p, (a, b) in enumerate([(0, 1), (1, 0)]):
        ref = oracle_pair(graphs, a, b)
        assert res["iters"][p] == ref.iters and base_status(res["status"][p]) == ref.status
        check_S(Ss[p], ref.S, "f64")
        check_margin(res["margin"][p], Ss[p], matches[p], "f64")


def test_large_invalid_and_degenerate(cf, ctx):
    graphs = _sizes_graphs([40, 50], seed=9)
    graphs.append(CFG(4, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([0.0, 0.0])))
    res, matches, Ss = _large(cf, ctx, graphs, [0, 7, 2, 0], [1, 0, 0, -1], "f32")
    assert res["status"][1] == cf.INVALID_INPUT and res["status"][3] == cf.INVALID_INPUT
    assert np.isnan(res["score"][1]) and res["iters"][1] == 0
    assert base_status(res["status"][2]) == cf.DEGENERATE and res["iters"][2] == 0
    ref = oracle_pair(graphs, 2, 0)
    assert ref.status == oracle.DEGENERATE
    check_S(Ss[2], ref.S, "f32")
    check_matching(Ss[2], matches[2], ref.S, "f32")
    assert res["margin"][2] == 0.0 and res["status"][2] & cf.NEAR_TIE  # every entry of S_0 ties
    ref0 = oracle_pair(graphs, 0, 1)
    er = check_S(Ss[0], ref0.S, "f32")
    check_margin(res["margin"][0], Ss[0], matches[0], "f32")
    check_matching(Ss[0], matches[0], ref0.S, "f32", er)


def test_large_replay_deterministic(cf, ctx):
    graphs = _sizes_graphs([300, 200, 150, 260], seed=3)
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, np.array([0, 2], np.int32), np.array([1, 3], np.int32), dtype="f32", want_S=True,
                 path="large")
    b.run()
    torch.cuda.synchronize()
    r1, S1 = b.results().tobytes(), b.S.clone()
    for _ in range(2):
        b.res.zero_()
        b.S.zero_()
        b.run()
        torch.cuda.synchronize()
        assert b.results().tobytes() == r1
        assert torch.equal(b.S, S1)


def test_large_agrees_with_batched_path(cf, ctx):
    graphs = _sizes_graphs([20, 33, 64, 100, 128], seed=4)
    pa, pb = np.triu_indices(len(graphs), k=1)
    gs = cf.pack(ctx, graphs)
    rb, mb, Sb = cf.score_batch(ctx, gs, pa.astype(np.int32), pb.astype(np.int32), dtype="f64", want_S=True)
    rl, ml, Sl = cf.score_batch(ctx, gs, pa.astype(np.int32), pb.astype(np.int32), dtype="f64", want_S=True,
                                path="large")
    assert np.array_equal(rb["iters"], rl["iters"]) and np.array_equal(rb["status"], rl["status"])
    for p in range(len(pa)):
        assert np.max(np.abs(Sl[p] - Sb[p])) <= 1e-12 * np.max(Sb[p])
        assert np.array_equal(ml[p], mb[p])


def test_large_fp32_workload2_pair_full_oracle(cf, ctx):
    """One pair of the large-pair workload (1151 x 1053), FP32, oracle in full."""
    w = config_graphs(2, scale=1 / 64)
    g = w["graphs"]
    res, matches, Ss = _large(cf, ctx, g, w["pair_a"], w["pair_b"], "f32")
    ga, gb = g[0], g[1]
    A = oracle.transition_matrix_sparse(ga.n, ga.src, ga.dst, ga.count)
    B = oracle.transition_matrix_sparse(gb.n, gb.src, gb.dst, gb.count)
    ref = oracle.score_pair(A, B, 200, 1e-12)
    er = check_S(Ss[0], ref.S, "f32")
    check_margin(res["margin"][0], Ss[0], matches[0], "f32")
    check_matching(Ss[0], matches[0], ref.S, "f32", er)
    assert res["iters"][0] == ref.iters and base_status(res["status"][0]) == ref.status


def test_large_workload2_full_launch(cf, ctx):
    """All 64 pairs (512-2048 nodes) in one call: every pair served, properties
    of every pair, and two pairs against stored oracle results."""
    w = config_graphs(2)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_S=True, path="large")
    b.run()
    torch.cuda.synchronize()
    res = b.results()
    assert len(res) == 64 and np.all(res["status"] != cf.INVALID_INPUT)
    nmin = np.minimum(b.nA, b.nB)
    assert np.all(res["score"] > 0) and np.all(res["score"] <= np.sqrt(nmin) + 1e-4)
    Ss, ms = b.S_list(), b.matches()
    gold = np.load(GOLDEN)
    for p in gold["pairs"]:
        p = int(p)
        S = Ss[p].astype(np.float64)
        assert S.shape == tuple(gold[f"p{p}_shape"])
        score, nu, delta, iters, status = gold[f"p{p}_meta"]
        assert res["iters"][p] == iters and base_status(res["status"][p]) == status
        idx, val = gold[f"p{p}_idx"], gold[f"p{p}_val"]
        est = np.sqrt(np.sum((S.reshape(-1)[idx] - val) ** 2) * S.size / idx.size)  # ||S_ref|| = 1
        assert est <= 1e-5, (p, est)
        assert abs(np.linalg.norm(S) - 1.0) <= 1e-5
        own, _ = oracle.greedy_match(S)
        assert np.array_equal(ms[p], own)
        # FP32 near ties may reorder picks; the score stays within 1e-4 relative
        assert abs(res["score"][p] - score) <= 1e-4 * score, (p, res["score"][p], score)
