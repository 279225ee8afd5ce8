"""Parity of the optimal-assignment matching (cfsim_assign) with the FP64
oracle.  Both run the Hungarian method with the same FP64 operations in the
same order and the same tie rule (smallest column), so the matchings must be
identical on the same S, ties included; the score (a sum the kernel adds in
another order) must agree to 1e-13 relative and equal the optimum of scipy's
solver.  The S matrices come from random draws (with exact ties) and from
the similarity kernels' own outputs."""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle
from cfgsynth import config_graphs

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


def _check(S, match, score):
    S64 = np.asarray(S, np.float64)
    want, wscore = oracle.optimal_assignment(S64)
    assert np.array_equal(match, want), (S.shape, match, want)
    assert abs(score - wscore) <= 1e-13 * max(1.0, abs(wscore))
    r, c = linear_sum_assignment(S64, maximize=True)
    assert abs(score - S64[r, c].sum()) <= 1e-12 * max(1.0, abs(wscore))


SHAPES = [(1, 1), (1, 7), (7, 1), (5, 5), (6, 9), (9, 6), (40, 40), (33, 70), (70, 33), (64, 65), (65, 64),
          (128, 128), (200, 150)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_random_and_tied_matrices(cf, ctx, dtype):
    rng = np.random.default_rng(1)
    mats = [rng.random(s) for s in SHAPES]
    mats += [rng.integers(0, 4, size=s).astype(np.float64) for s in [(8, 8), (12, 20), (20, 12), (64, 64)]]
    mats += [np.ones((5, 9)), np.zeros((3, 3))]
    if dtype == "f32":
        mats = [m.astype(np.float32) for m in mats]
    matches, scores = cf.assign(ctx, mats, dtype)
    for S, m, s in zip(mats, matches, scores):
        _check(S, m, s)


def test_non_finite_matrix_is_marked_and_others_are_unaffected(cf, ctx):
    rng = np.random.default_rng(2)
    mats = [rng.random((6, 6)), rng.random((5, 8)), rng.random((7, 4))]
    mats[1][2, 3] = np.nan
    mats[2][0, 0] = np.inf
    matches, scores = cf.assign(ctx, mats, "f64")
    _check(mats[0], matches[0], scores[0])
    for k in (1, 2):
        assert np.isnan(scores[k]) and (matches[k] == -1).all()


def test_similarity_batch_and_determinism(cf, ctx):
    w = config_graphs(1, scale=20 / 256)
    gs = cf.pack(ctx, w["graphs"])
    for path, kw in (("batch", {}), ("damped", dict(alpha=0.85))):
        b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_S=True, path=path, **kw)
        b.run()
        m1, s1 = b.assign()
        m2, s2 = b.assign()
        torch.cuda.synchronize()
        assert torch.equal(m1, m2) and torch.equal(s1, s2)
        Ss, res = b.S_list(), b.results()
        m1 = m1.cpu().numpy()
        s1 = s1.cpu().numpy()
        for p in range(b.n_pairs):
            o, n = b.match_off_h[p], b.nB[p]
            _check(Ss[p], m1[o:o + n], s1[p])
            # the optimum is at least the greedy total
            assert s1[p] >= res[p]["score"] * (1 - 1e-6)


def test_full_all_pairs_workload_sampled(cf, ctx):
    """All 32,640 pairs of the 256-CFG workload (FP32 S from the batched
    path), as the benchmark runs it; 24 seeded pairs against the oracle."""
    w = config_graphs(1)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_S=True)
    b.run()
    m, s = b.assign()
    torch.cuda.synchronize()
    s = s.cpu().numpy()
    m = m.cpu().numpy()
    assert np.isfinite(s).all()
    res = b.results()
    assert (s >= res["score"] * (1 - 1e-6)).all()
    rng = np.random.default_rng(170702423)
    S_all = b.S.cpu().numpy()
    for p in rng.choice(b.n_pairs, size=24, replace=False):
        nA, nB = b.nA[p], b.nB[p]
        S = S_all[b.S_off_h[p]:b.S_off_h[p] + nA * nB].reshape(nB, nA)
        o = b.match_off_h[p]
        _check(S, m[o:o + nB], s[p])
