"""Parity of the HIP path (through the C ABI) with the FP64 oracle."""
import numpy as np
import pytest

import oracle
from cfgsynth import CFG, Grammar, config_graphs, make_cfg
from tests.parity import (FP64_FINAL, NEAR_TIE, base_status, chain_depth, check_margin, check_matching, check_S,
                          oracle_pair, rel_err, stop_drift)

TIE_TOL = {"f64": 1e-12, "f32": 2e-5}

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


def _g(n, edges):
    e = np.asarray(edges, np.float64).reshape(-1, 3)
    return CFG(n, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.float64))


def _dense_from_set(gs, g):
    rp, col, w = gs.host_csr(g)
    n = len(rp) - 1
    M = np.zeros((n, n))
    for u in range(n):
        for p in range(rp[u], rp[u + 1]):
            M[u, col[p]] += w[p]
    return M


# ------------------------------------------------------------------ a1
def test_pack_equals_oracle_transition_matrices(cf, ctx):
    graphs = config_graphs(1, scale=16 / 256)["graphs"] + [
        _g(4, [[0, 1, 5], [0, 1, 3], [0, 2, 0], [1, 3, 7], [2, 3, 1]]),   # repeated jump, zero count
        _g(3, []),                                                       # no jumps at all
        _g(1, [[0, 0, 9]]),                                              # single self-loop node
        _g(6, [[0, 5, 1], [1, 5, 2], [2, 5, 3], [3, 5, 4], [4, 5, 5], [0, 1, 1]]),
    ]
    gs = cf.pack(ctx, graphs)
    for g, G in enumerate(graphs):
        ref = oracle.transition_matrix(G.n, G.src, G.dst, G.count)
        np.testing.assert_array_equal(_dense_from_set(gs, g), ref, err_msg=f"graph {g}")
    # CSC lists are the transposed CSR, sorted, with eid pointing at the CSR entry
    cp, row, eid = gs.col_ptr.cpu().numpy(), gs.row.cpu().numpy(), gs.eid.cpu().numpy()
    rp, col = gs.row_ptr.cpu().numpy(), gs.col.cpu().numpy()
    for g in range(len(graphs)):
        n0, e0 = int(gs.node_off[g]), int(gs.edge_off[g])
        n = int(gs.node_off[g + 1]) - n0
        for v in range(n):
            b, e = cp[n0 + g + v], cp[n0 + g + v + 1]
            rows = row[e0 + b:e0 + e]
            assert list(rows) == sorted(rows)
            for t in range(b, e):
                p = eid[e0 + t]
                assert col[e0 + p] == v
                u = row[e0 + t]
                assert rp[n0 + g + u] <= p < rp[n0 + g + u + 1]


def test_pack_flags_bad_input(cf, ctx):
    bad = [_g(3, [[0, 1, 1], [1, 7, 1]]), _g(2, [[0, 1, float("nan")]]), _g(2, [[0, 1, -2.0]])]
    for G, flag, code in zip(bad, [1, 2, 4], [-2, -3, -4]):
        # the host check refuses the lists before anything is uploaded ...
        with pytest.raises(cf.CfsimError) as e:
            cf.pack(ctx, [G])
        assert e.value.code == code
        # ... and the device pack flags them in err_flags when the host check is skipped
        gs = cf.pack(ctx, [G], check=False)
        assert gs is not None
    from paper_1707_02423_amd import cfsim as cfm
    import ctypes
    for G, flag in zip(bad, [1, 2, 4]):
        node_off, edge_off, src, dst, cnt = cfm.concat_coo([G])
        t = lambda a, dt: torch.as_tensor(a, dtype=dt).cuda()
        n, m = int(node_off[-1]), int(edge_off[-1])
        outs = [torch.empty(n + 1, dtype=torch.int32, device="cuda"), torch.empty(m, dtype=torch.int32, device="cuda"),
                torch.empty(m, dtype=torch.float64, device="cuda"), torch.empty(n + 1, dtype=torch.int32, device="cuda"),
                torch.empty(m, dtype=torch.int32, device="cuda"), torch.empty(m, dtype=torch.int32, device="cuda")]
        err = torch.zeros(1, dtype=torch.int32, device="cuda")
        ws_b = cfm.lib().cfsim_pack_workspace_size(1, n, m)
        ws = torch.empty(max(ws_b, 1), dtype=torch.uint8, device="cuda")
        ins = [t(node_off, torch.int64), t(edge_off, torch.int64), t(src, torch.int32), t(dst, torch.int32),
               t(cnt, torch.float64)]
        rc = cfm.lib().cfsim_pack(ctx.handle, 1, n, m, *[x.data_ptr() for x in ins], *[x.data_ptr() for x in outs],
                                  err.data_ptr(), ws.data_ptr(), ws_b, None)
        assert rc == 0
        torch.cuda.synchronize()
        assert int(err.item()) & flag


# ------------------------------------------------------------------ plain path
def _plain_case(cf, ctx, graphs, a, b, dtype, max_iter=200, tol=1e-12):
    gs = cf.pack(ctx, graphs)
    got = cf.score(ctx, gs, a, b, dtype=dtype, max_iter=max_iter, tol=tol)
    ref = oracle_pair(graphs, a, b, max_iter, tol)
    er = check_S(got["S"], ref.S, dtype, max(got["iters"], ref.iters), chain_depth(graphs[a], graphs[b]),
                 stop_drift(graphs, a, b, got["iters"], ref.iters))
    assert got["iters"] == ref.iters and base_status(got["status"]) == ref.status
    check_margin(got["margin"], got["S"], got["match"], dtype)
    assert bool(got["status"] & NEAR_TIE) == (got["margin"] <= TIE_TOL[dtype])
    assert abs(got["nu"] - ref.nu) <= (1e-9 if dtype == "f64" else 1e-5) * max(1.0, ref.nu)
    # the kernels take the even-step change from running sums (no stored S_{k-2});
    # it must agree with the oracle's direct ||S_k - S_{k-2}||
    if np.isfinite(ref.delta):
        dtol = 1e-9 * ref.delta + 1e-14 if dtype == "f64" else 1e-5
        assert abs(got["delta"] - ref.delta) <= dtol, (got["delta"], ref.delta)
    else:
        assert got["delta"] == float("inf")
    check_matching(got["S"], got["match"], ref.S, dtype, er)
    S64 = got["S"].astype(np.float64)
    assert abs(got["score"] - sum(S64[i, j] for i, j in enumerate(got["match"]) if j >= 0)) < 1e-12
    return got, ref


def test_plain_fp64_workload0(cf, ctx):
    w = config_graphs(0)
    got, ref = _plain_case(cf, ctx, w["graphs"], 0, 1, "f64")
    assert abs(got["score"] - ref.score) < 1e-9


@pytest.mark.parametrize("nA,nB", [(2, 2), (5, 9), (9, 5), (16, 16), (40, 7), (7, 40), (64, 64), (65, 30),
                                   (30, 65), (90, 60), (128, 3)])
def test_plain_fp64_sizes(cf, ctx, nA, nB):
    rng = np.random.default_rng(nA * 1000 + nB)
    graphs = [make_cfg(nA, Grammar(counts="trip"), rng), make_cfg(nB, Grammar(counts="trip"), rng)]
    _plain_case(cf, ctx, graphs, 0, 1, "f64")


@pytest.mark.parametrize("nA,nB", [(12, 16), (64, 100), (128, 128), (20, 200), (200, 20)])
def test_plain_fp32_sizes(cf, ctx, nA, nB):
    rng = np.random.default_rng(nA * 7 + nB)
    graphs = [make_cfg(nA, Grammar(counts="trip"), rng), make_cfg(nB, Grammar(counts="trip"), rng)]
    _plain_case(cf, ctx, graphs, 0, 1, "f32")


@pytest.mark.parametrize("max_iter,tol", [(1, 1e-12), (7, 0.0), (33, 1e-12), (200, 1e-3), (200, 0.0)])
def test_plain_iteration_controls(cf, ctx, max_iter, tol):
    rng = np.random.default_rng(3)
    graphs = [make_cfg(14, Grammar(), rng), make_cfg(11, Grammar(), rng)]
    got, ref = _plain_case(cf, ctx, graphs, 0, 1, "f64", max_iter, tol)
    if max_iter == 1:
        assert got["delta"] == float("inf")


# The matching runs three ways: sorted rows walked in registers (at most 256
# stored rows), the same walk with its state in LDS (more rows), and rounds of
# mutual bests (stored rows over 256 entries).  Stored orientation: (60, 300)
# keeps 300 rows of 60, (300, 250) stores 300 rows of 250, (600, 10) 10 rows
# of 600 (global kernel).
@pytest.mark.parametrize("nA,nB", [(60, 300), (300, 250), (600, 10)])
def test_plain_matching_paths(cf, ctx, nA, nB):
    rng = np.random.default_rng(nA + 17 * nB)
    graphs = [make_cfg(nA, Grammar(counts="trip"), rng), make_cfg(nB, Grammar(counts="trip"), rng)]
    got, ref = _plain_case(cf, ctx, graphs, 0, 1, "f64", max_iter=60)
    own, _ = oracle.greedy_match(got["S"].astype(np.float64))
    assert np.array_equal(got["match"], own)

def test_plain_oscillating_pair_converges_on_even_step(cf, ctx):
    path = _g(3, [[0, 1, 1], [1, 2, 1]])
    loop = _g(1, [[0, 0, 1]])
    got, ref = _plain_case(cf, ctx, [path, loop], 0, 1, "f64")
    assert got["iters"] == 2 and base_status(got["status"]) == cf.CONVERGED


def test_plain_degenerate_pair(cf, ctx):
    graphs = [make_cfg(6, Grammar(), seed=1), _g(4, [])]
    gs = cf.pack(ctx, graphs)
    got = cf.score(ctx, gs, 0, 1, dtype="f64")
    # every entry of S_0 ties: the margin is 0
    assert got["status"] == cf.DEGENERATE | cf.NEAR_TIE and got["iters"] == 0 and got["margin"] == 0.0
    np.testing.assert_allclose(got["S"], np.full((4, 6), 1 / np.sqrt(24)), rtol=1e-15)
    assert got["match"].tolist() == [0, 1, 2, 3]


def test_plain_long_lists_use_overflow_path(cf, ctx):
    # node 0 fans out to 6 nodes and node 7 collects 7 predecessors
    fan = _g(8, [[0, k, k] for k in range(1, 7)] + [[k, 7, 1] for k in range(0, 7)] + [[7, 0, 2]])
    other = make_cfg(30, Grammar(), seed=5)
    _plain_case(cf, ctx, [fan, other], 0, 1, "f64")
    _plain_case(cf, ctx, [other, fan], 0, 1, "f64")
    _plain_case(cf, ctx, [fan, fan], 0, 1, "f32")


def test_plain_pair_determinism(cf, ctx):
    graphs = config_graphs(1, scale=2 / 256)["graphs"]
    gs = cf.pack(ctx, graphs)
    r1 = cf.score(ctx, gs, 0, 1, dtype="f32")
    r2 = cf.score(ctx, gs, 0, 1, dtype="f32")
    assert np.array_equal(r1["S"], r2["S"]) and r1["score"] == r2["score"]


# ------------------------------------------------------------------ batched path
def _batch_check(cf, ctx, graphs, pa, pb, dtype, sample=None, max_iter=200, tol=1e-12):
    gs = cf.pack(ctx, graphs)
    res, matches, Ss = cf.score_batch(ctx, gs, pa, pb, dtype=dtype, max_iter=max_iter, tol=tol, want_S=True)
    idx = range(len(pa)) if sample is None else sample
    worst, near = 0.0, 0
    for p in idx:
        assert res["status"][p] != cf.INVALID_INPUT, f"pair {p} refused"
        ref = oracle_pair(graphs, int(pa[p]), int(pb[p]), max_iter, tol)
        er = check_S(Ss[p], ref.S, dtype, max(res["iters"][p], ref.iters), chain_depth(graphs[pa[p]], graphs[pb[p]]),
                     stop_drift(graphs, pa[p], pb[p], res["iters"][p], ref.iters))
        worst = max(worst, rel_err(Ss[p], ref.S))
        assert base_status(res["status"][p]) == ref.status or dtype == "f32", f"pair {p} status"
        if dtype == "f64":
            assert res["iters"][p] == ref.iters
        check_margin(res["margin"][p], Ss[p], matches[p], dtype)
        assert bool(res["status"][p] & NEAR_TIE) == (res["margin"][p] <= TIE_TOL[dtype])
        near += check_matching(Ss[p], matches[p], ref.S, dtype, er) == "near-tie"
        S64 = Ss[p].astype(np.float64)
        assert abs(res["score"][p] - sum(S64[i, j] for i, j in enumerate(matches[p]) if j >= 0)) < 1e-12
    return res, worst, near


def test_batch_fp32_workload1_subset(cf, ctx):
    w = config_graphs(1, scale=22 / 256)
    res, worst, near = _batch_check(cf, ctx, w["graphs"], w["pair_a"], w["pair_b"], "f32")
    assert len(res) == 231
    assert np.all(res["iters"] <= 200)


def test_batch_fp64_workload1_subset(cf, ctx):
    w = config_graphs(1, scale=12 / 256)
    _batch_check(cf, ctx, w["graphs"], w["pair_a"], w["pair_b"], "f64")


def test_batch_mixed_sizes_every_variant(cf, ctx):
    rng = np.random.default_rng(11)
    sizes = [1, 2, 3, 8, 16, 17, 33, 64, 65, 100, 127, 128, 150, 200]
    graphs = [make_cfg(n, Grammar(counts="trip"), rng) if n >= 2 else _g(1, [[0, 0, 3]]) for n in sizes]
    pa, pb = np.triu_indices(len(graphs), k=0)
    pa, pb = pa.astype(np.int32), pb.astype(np.int32)
    gs = cf.pack(ctx, graphs)
    res, matches, Ss = cf.score_batch(ctx, gs, pa, pb, dtype="f32", want_S=True)
    assert np.all(res["status"] != cf.INVALID_INPUT), "every pair must be served (LDS or global kernel)"
    for p in range(len(pa)):
        nA, nB = sizes[pa[p]], sizes[pb[p]]
        ref = oracle_pair(graphs, int(pa[p]), int(pb[p]))
        er = check_S(Ss[p], ref.S, "f32", max(res["iters"][p], ref.iters), chain_depth(graphs[pa[p]], graphs[pb[p]]),
                     stop_drift(graphs, pa[p], pb[p], res["iters"][p], ref.iters))
        check_margin(res["margin"][p], Ss[p], matches[p], "f32")
        check_matching(Ss[p], matches[p], ref.S, "f32", er)


def test_batch_invalid_indices_and_empty(cf, ctx):
    graphs = config_graphs(1, scale=3 / 256)["graphs"]
    gs = cf.pack(ctx, graphs)
    pa = np.array([0, 5, -1, 1], np.int32)
    pb = np.array([1, 0, 2, 2], np.int32)
    res, matches, _ = cf.score_batch(ctx, gs, pa, pb, dtype="f32", want_match=False)
    assert res["status"][1] == cf.INVALID_INPUT and res["status"][2] == cf.INVALID_INPUT
    assert base_status(res["status"][0]) in (cf.CONVERGED, cf.HIT_MAX_ITER)
    r0, _, _ = cf.score_batch(ctx, gs, np.zeros(0, np.int32), np.zeros(0, np.int32), want_match=False)
    assert len(r0) == 0


def test_batch_deterministic_and_graph_replay(cf, ctx):
    w = config_graphs(1, scale=10 / 256)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_S=True)
    b.run()
    torch.cuda.synchronize()
    r1, S1 = b.results().copy(), b.S.clone()
    for _ in range(3):   # replays of the cached graph, with host syncs between
        b.res.zero_()
        b.run()
        torch.cuda.synchronize()
        assert np.array_equal(b.results(), r1)
        assert torch.equal(b.S, S1)


def test_batch_matches_plain_path(cf, ctx):
    # the plain path may run a pair on a larger kernel than the batch (its
    # norms then sum over another number of waves): FP64 rounding apart, the
    # same S, update count and matching
    w = config_graphs(1, scale=6 / 256)
    gs = cf.pack(ctx, w["graphs"])
    res, matches, Ss = cf.score_batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f64", want_S=True)
    for p in range(len(res)):
        r = cf.score(ctx, gs, int(w["pair_a"][p]), int(w["pair_b"][p]), dtype="f64")
        assert np.max(np.abs(r["S"] - Ss[p])) <= 1e-13 * np.max(Ss[p])
        assert r["iters"] == res["iters"][p]
        if not (res["status"][p] & NEAR_TIE):
            assert np.array_equal(r["match"], matches[p])


def test_workload1_full_size_sampled(cf, ctx):
    """The benchmark launch (256 graphs, 32,640 pairs, FP32): properties of
    every pair, oracle parity on a seeded sample."""
    w = config_graphs(1)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_S=True)
    b.run()
    torch.cuda.synchronize()
    res = b.results()
    assert len(res) == 32640
    assert np.all(res["status"] != cf.INVALID_INPUT)
    assert np.all(np.isfinite(res["score"])) and np.all(res["nu"] > 0)
    nmin = np.minimum(b.nA, b.nB)
    assert np.all(res["score"] > 0) and np.all(res["score"] <= np.sqrt(nmin) + 1e-5)
    rng = np.random.default_rng(2024)
    sample = rng.choice(len(res), size=24, replace=False)
    S_all = b.S
    for p in sample:
        o, nA, nB = int(b.S_off_h[p]), int(b.nA[p]), int(b.nB[p])
        S = S_all[o:o + nA * nB].cpu().numpy().reshape(nB, nA)
        assert abs(np.linalg.norm(S.astype(np.float64)) - 1) < 1e-5
        ga, gb = int(w["pair_a"][p]), int(w["pair_b"][p])
        ref = oracle_pair(w["graphs"], ga, gb)
        er = check_S(S, ref.S, "f32", max(res["iters"][p], ref.iters), chain_depth(w["graphs"][ga], w["graphs"][gb]),
                     stop_drift(w["graphs"], ga, gb, res["iters"][p], ref.iters))
        m = b.match[int(b.match_off_h[p]):int(b.match_off_h[p]) + nB].cpu().numpy()
        check_margin(res["margin"][p], S, m, "f32")
        check_matching(S, m, ref.S, "f32", er)


def test_batch_buckets_and_timed_launch(cf, ctx):
    rng = np.random.default_rng(12)
    sizes = [4, 16, 40, 70, 100, 128, 200]
    graphs = [make_cfg(n, Grammar(counts="trip"), rng) for n in sizes]
    pa, pb = np.triu_indices(len(graphs), k=0)
    pa = np.concatenate([pa, [0, 99]]).astype(np.int32)
    pb = np.concatenate([pb, [-3, 1]]).astype(np.int32)
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, pa, pb, dtype="f32", want_S=True)
    bk = b.buckets()
    assert bk.shape == (len(pa),) and np.all((bk >= 0) & (bk < cf.NUM_BUCKETS))
    assert bk[-1] == 6 and bk[-2] == 6 and np.all(bk[:-2] != 6)
    # larger pairs never land in a smaller bucket than a smaller pair of the same shape class
    area = np.array([sizes[a] * sizes[c] for a, c in zip(pa[:-2], pb[:-2])])
    assert bk[:-2][np.argmax(area)] >= bk[:-2][np.argmin(area)]
    b.run()
    torch.cuda.synchronize()
    r_graph, S_graph = b.results().copy(), b.S.clone()
    ctx.set_timing(True)
    try:
        b.res.zero_()
        b.run()
        ms = ctx.batch_timings()
    finally:
        ctx.set_timing(False)
    assert b.results().tobytes() == r_graph.tobytes() and torch.equal(b.S, S_graph)
    used = np.unique(bk[bk < 6])
    assert ms.shape == (cf.NUM_BUCKETS,) and np.all(ms >= 0)
    assert np.all(ms[used] > 0), ms
    assert np.all(r_graph["status"][bk == 6] == cf.INVALID_INPUT)


# ------------------------------------------------------------------ FP64 pass of FP32 calls
def test_fp64_final_batch_replaces_near_ties(cf, ctx):
    """CFSIM_FLAG_FP64_FINAL: the near-tie pairs of an FP32 batch carry the
    FP64 results (bit for bit those of an FP64 batch), every other pair its
    FP32 result (bit for bit those of a plain FP32 batch)."""
    w = config_graphs(1, scale=20 / 256)
    gs = cf.pack(ctx, w["graphs"])
    pa, pb = w["pair_a"], w["pair_b"]
    r32, m32, S32 = cf.score_batch(ctx, gs, pa, pb, dtype="f32", want_S=True)
    r64, m64, S64 = cf.score_batch(ctx, gs, pa, pb, dtype="f64", want_S=True)
    rf, mf, Sf = cf.score_batch(ctx, gs, pa, pb, dtype="f32", want_S=True, fp64_final=True)
    near = (r32["status"] & NEAR_TIE) != 0
    assert near.any() and not near.all()
    assert np.array_equal((rf["status"] & FP64_FINAL) != 0, near)
    for p in range(len(pa)):
        if near[p]:
            for k in ("score", "nu", "delta", "margin", "iters", "status"):
                want = (r64[k][p] | FP64_FINAL) if k == "status" else r64[k][p]
                assert rf[k][p] == want, (p, k, rf[k][p], want)
            assert np.array_equal(mf[p], m64[p])
            assert np.array_equal(Sf[p], S64[p].astype(np.float32))
        else:
            assert rf[p].tobytes() == r32[p].tobytes()
            assert np.array_equal(mf[p], m32[p]) and np.array_equal(Sf[p], S32[p])
    # FP64-finalised pairs agree with the oracle's matching under the FP64 contract
    for p in np.flatnonzero(near)[:12]:
        ref = oracle_pair(w["graphs"], int(pa[p]), int(pb[p]))
        er = check_S(S64[p], ref.S, "f64")
        check_matching(S64[p], mf[p], ref.S, "f64", er)


def test_fp64_final_single_pair(cf, ctx):
    # two copies of one CFG: symmetric S, exact ties between mirrored entries
    g = make_cfg(24, Grammar(counts="trip"), seed=9)
    gs = cf.pack(ctx, [g, g, make_cfg(30, Grammar(counts="trip"), seed=10)])
    r32 = cf.score(ctx, gs, 0, 1, dtype="f32")
    rf = cf.score(ctx, gs, 0, 1, dtype="f32", fp64_final=True)
    r64 = cf.score(ctx, gs, 0, 1, dtype="f64")
    if r32["status"] & NEAR_TIE:
        assert rf["status"] == r64["status"] | FP64_FINAL
        assert rf["score"] == r64["score"] and np.array_equal(rf["match"], r64["match"])
        assert np.array_equal(rf["S"], r64["S"].astype(np.float32))
    else:
        assert rf["status"] == r32["status"] and np.array_equal(rf["S"], r32["S"])
    # a pair without a near tie keeps its FP32 result
    for a, b in ((0, 2), (2, 0)):
        q32 = cf.score(ctx, gs, a, b, dtype="f32")
        qf = cf.score(ctx, gs, a, b, dtype="f32", fp64_final=True)
        if not q32["status"] & NEAR_TIE:
            assert qf["status"] == q32["status"] and np.array_equal(qf["S"], q32["S"])
