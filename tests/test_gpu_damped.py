"""Parity of the damped IsoRank measure (Table 1, row "Iso", full form
(I - alpha Q x P) x = (1 - alpha) E with IsoRank's column-normalised
operator) with the FP64 oracle, through cfsim_score_damped.

Gates: FP64 S within 1e-10 element-wise (relative to max |S|), in relative
Frobenius norm and per entry (every entry is at least (1 - alpha) E > 0 for
the uniform prior, so relative per-entry errors are well defined), the same
update count and status, nu to 1e-12 relative and delta to 1e-14 absolute
(a sum of |x_k - x_{k-1}| over entries of size ~1/(n_A n_B), each formed
from two FP64 values one rounding away from the oracle's).  FP32 S within
1e-5 element-wise and in relative Frobenius norm (the tolerance FP32 results
are held to); the damped update is an affine contraction rather than a
projective one, so the per-entry relative FP32 error is measured and used
for the matching certificate, not gated on its own.  Matchings follow the
same contract as the undamped measure: equal to the oracle's greedy on the
GPU's own S, and equal to the oracle's matching unless the oracle's S has a
near tie (then certified)."""
import numpy as np
import pytest

import oracle
from cfgsynth import CFG, Grammar, config_graphs, make_cfg
from tests.parity import check_margin, check_matching, check_S, entry_rel_err, rel_err

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


def _tm(g):
    return oracle.transition_matrix(g.n, g.src, g.dst, g.count)


def _graphs(sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        if n == 1:
            out.append(CFG(1, np.array([0], np.int32), np.array([0], np.int32), np.array([3.0])))
        elif n == 0:   # one node, no jump: an all-zero matrix
            out.append(CFG(1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0)))
        else:
            out.append(make_cfg(n, Grammar(counts="trip"), rng))
    return out


def _check_pair(r, m, S, A, B, alpha, dtype, prior=None, max_iter=200, tol=1e-12):
    ref = oracle.score_pair_damped(A, B, alpha, prior, max_iter, tol)
    if dtype == "f64":
        check_S(S, ref.S, "f64")
        assert int(r["iters"]) == ref.iters, (int(r["iters"]), ref.iters)
        assert int(r["status"]) & 15 == ref.status
        assert abs(r["nu"] - ref.nu) <= 1e-12 * ref.nu
        assert abs(r["delta"] - ref.delta) <= 1e-14
    else:
        Sd, R = np.asarray(S, np.float64), ref.S
        assert float(np.max(np.abs(Sd - R))) <= 1e-5 * float(np.max(R))
        assert rel_err(Sd, R) <= 1e-5
    check_margin(r["margin"], S, m, dtype)
    kind = check_matching(S, m, ref.S, dtype, entry_err=entry_rel_err(S, ref.S, dtype))
    score = float(np.sum([S[i, j] for i, j in enumerate(m) if j >= 0], dtype=np.float64))
    assert abs(r["score"] - score) <= 1e-12 * max(1.0, score)
    return kind


@pytest.mark.parametrize("alpha", [0.0, 0.5, 0.85, 0.95])
def test_fp64_ragged_sizes_match_the_oracle(cf, ctx, alpha):
    sizes = [1, 0, 2, 5, 12, 63, 64, 65, 100, 128, 17, 129, 40]
    graphs = _graphs(sizes, 7)
    pa = np.array([0, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 3, 1, 9], np.int32)
    pb = np.array([2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 4, 3, 9, 12], np.int32)
    gs = cf.pack(ctx, graphs)
    res, matches, Ss = cf.score_damped(ctx, gs, pa, pb, alpha=alpha, dtype="f64", want_S=True)
    mats = [_tm(g) for g in graphs]
    for p, (a, b) in enumerate(zip(pa, pb)):
        _check_pair(res[p], matches[p], Ss[p], mats[a], mats[b], alpha, "f64")


def test_fp32_batch_matches_the_oracle(cf, ctx):
    w = config_graphs(1, scale=24 / 256)
    graphs, pa, pb = w["graphs"], w["pair_a"], w["pair_b"]
    gs = cf.pack(ctx, graphs)
    res, matches, Ss = cf.score_damped(ctx, gs, pa, pb, alpha=0.85, dtype="f32", want_S=True)
    mats = [_tm(g) for g in graphs]
    rng = np.random.default_rng(5)
    kinds = []
    for p in rng.choice(len(pa), size=40, replace=False):
        a, b = pa[p], pb[p]
        kinds.append(_check_pair(res[p], matches[p], Ss[p], mats[a], mats[b], 0.85, "f32"))
    assert kinds.count("exact") >= 30
    # every pair: unit norm, positive entries, a finite score
    for p in range(len(pa)):
        assert abs(np.linalg.norm(Ss[p].astype(np.float64)) - 1.0) <= 1e-5
        assert Ss[p].min() > 0 and np.isfinite(res[p]["score"])


def test_user_priors_and_invalid_priors(cf, ctx):
    graphs = _graphs([6, 9, 30, 70, 11], 11)
    pa = np.array([0, 1, 2, 3, 4, 0, 2], np.int32)
    pb = np.array([1, 2, 3, 4, 0, 3, 4], np.int32)
    gs = cf.pack(ctx, graphs)
    rng = np.random.default_rng(3)
    priors = []
    for a, b in zip(pa, pb):
        P = rng.random((graphs[b].n, graphs[a].n)) * (rng.random((graphs[b].n, graphs[a].n)) < 0.7)
        P[0, 0] = 2.0
        priors.append(P)
    priors[4] = -priors[4]          # negative
    priors[5] = np.zeros_like(priors[5])
    priors[6] = priors[6].copy()
    priors[6][1, 1] = np.nan
    res, matches, Ss = cf.score_damped(ctx, gs, pa, pb, alpha=0.7, prior=priors, dtype="f64", want_S=True)
    mats = [_tm(g) for g in graphs]
    for p in range(4):
        _check_pair(res[p], matches[p], Ss[p], mats[pa[p]], mats[pb[p]], 0.7, "f64", prior=priors[p])
    for p in (4, 5, 6):
        assert res[p]["status"] == cf.INVALID_INPUT and np.isnan(res[p]["score"])


def test_fp64_pairs_beyond_lds_take_the_global_kernel(cf, ctx):
    graphs = _graphs([200, 150, 90], 21)
    pa = np.array([0, 1], np.int32)
    pb = np.array([1, 2], np.int32)
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, pa, pb, dtype="f64", want_S=True, path="damped", alpha=0.85)
    assert b.buckets()[0] == cf.NUM_BUCKETS - 2   # the global-memory kernel
    b.run()
    torch.cuda.synchronize()
    res, matches, Ss = b.results(), b.matches(), b.S_list()
    mats = [_tm(g) for g in graphs]
    for p, (a, bb) in enumerate(zip(pa, pb)):
        _check_pair(res[p], matches[p], Ss[p], mats[a], mats[bb], 0.85, "f64")


def test_replays_are_bit_identical(cf, ctx):
    w = config_graphs(1, scale=12 / 256)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_S=True, path="damped", alpha=0.85)
    b.run()
    torch.cuda.synchronize()
    r0, S0, m0 = b.results().copy(), b.S.clone(), b.match.clone()
    b.run()
    torch.cuda.synchronize()
    assert np.array_equal(b.results().view(np.uint8), r0.view(np.uint8))
    assert torch.equal(b.S, S0) and torch.equal(b.match, m0)


def test_full_all_pairs_workload_sampled_against_the_oracle(cf, ctx):
    """The 32,640-pair workload (256 CFGs, n ~ U[8,128]) in FP32 with the
    launch configuration the benchmark times; 16 seeded pairs are checked
    against the oracle, every pair for its invariants."""
    w = config_graphs(1)
    graphs, pa, pb = w["graphs"], w["pair_a"], w["pair_b"]
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, pa, pb, dtype="f32", want_S=False, path="damped", alpha=0.85)
    b.run()
    torch.cuda.synchronize()
    res = b.results()
    assert not (res["status"] & cf.INVALID_INPUT).any()
    assert np.isfinite(res["score"]).all() and (res["score"] > 0).all()
    rng = np.random.default_rng(170702423)
    sample = rng.choice(len(pa), size=16, replace=False)
    sub = cf.Batch(ctx, gs, pa[sample], pb[sample], dtype="f32", want_S=True, path="damped", alpha=0.85)
    sub.run()
    torch.cuda.synchronize()
    rs, ms, Ss = sub.results(), sub.matches(), sub.S_list()
    for q, p in enumerate(sample):
        assert rs[q]["score"] == res[p]["score"]   # same kernels, same pair: same result
        _check_pair(rs[q], ms[q], Ss[q], _tm(graphs[pa[p]]), _tm(graphs[pb[p]]), 0.85, "f32")
