"""Parity of the elementwise distances (Table 1: Euclidean, Manhattan,
Minkowski, Jaccard, Cosine between the pair's transition matrices at the
common size of Sections 4 and 4.1) with the FP64 oracle, through
cfsim_distances.

Gate: each distance is built from six sums of n = M^2 non-negative FP64
terms that the kernel adds in another order than numpy; the error of such a
sum is at most (n - 1) u of the sum of its terms (u = 2^-53), each term is
within a few u of the oracle's (the interpolated entry has at most four
products), and the square root, quotient and p-th root add a few u more.
So every distance but Cosine is held to a relative error of
4 (n + 16) u, and Cosine (1 - c with 0 <= c <= 1) to that absolute error.
"""
import numpy as np
import pytest

import oracle
from cfgsynth import CFG, Grammar, config_graphs, make_cfg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = 2.0 ** -53


@pytest.fixture(scope="module")
def cf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02423_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(cf):
    return cf.Context(0)


def _matrix(g: CFG):
    return oracle.transition_matrix_sparse(g.n, g.src, g.dst, g.count) if g.n > 400 else \
        oracle.transition_matrix(g.n, g.src, g.dst, g.count)


def check_distances(got, graphs, pa, pb, p, mats=None):
    """Compare every listed pair's five distances with the oracle."""
    mats = {} if mats is None else mats
    worst = 0.0
    for q, (a, b) in enumerate(zip(pa, pb)):
        for g in (a, b):
            if g not in mats:
                mats[g] = _matrix(graphs[g])
        want = oracle.pair_distances(mats[a], mats[b], p)
        M = max(graphs[a].n, graphs[b].n)
        gate = 4.0 * (M * M + 16) * U
        for k in range(4):
            err = abs(got[q, k] - want[k])
            assert err <= gate * abs(want[k]) or (want[k] == 0.0 and got[q, k] == 0.0), (q, a, b, k, got[q, k], want[k])
            if want[k] > 0:
                worst = max(worst, err / want[k])
        if np.isnan(want[4]):
            assert np.isnan(got[q, 4]), (q, a, b)
        else:
            assert abs(got[q, 4] - want[4]) <= gate, (q, a, b, got[q, 4], want[4])
    return worst


def _graphs(sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        if n == 1:
            out.append(CFG(1, np.array([0], np.int32), np.array([0], np.int32), np.array([3.0])))
        elif n == 0:   # a single node without edges: an all-zero matrix
            out.append(CFG(1, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0)))
        else:
            out.append(make_cfg(n, Grammar(counts="trip"), rng))
    return out


SIZES = [0, 1, 2, 3, 5, 8, 13, 31, 45, 46, 63, 64, 65, 100, 128, 129, 200, 333]


@pytest.fixture(scope="module")
def small(cf, ctx):
    graphs = _graphs(SIZES, seed=2024)
    gs = cf.pack(ctx, graphs)
    a, b = np.triu_indices(len(graphs), k=0)      # every unordered pair and every self pair
    return graphs, gs, a.astype(np.int32), b.astype(np.int32)


@pytest.mark.parametrize("p", [3.0, 1.0, 2.5])
def test_small_pairs_match_the_oracle(cf, ctx, small, p):
    graphs, gs, a, b = small
    got = cf.distances(ctx, gs, a, b, p=p).cpu().numpy()
    check_distances(got, graphs, a, b, p)


def test_swapped_pairs_are_identical_and_self_pairs_zero(cf, ctx, small):
    graphs, gs, a, b = small
    d_ab = cf.distances(ctx, gs, a, b).cpu().numpy()
    d_ba = cf.distances(ctx, gs, b, a).cpu().numpy()
    np.testing.assert_array_equal(d_ab, d_ba)
    self_pairs = a == b
    assert np.all(d_ab[self_pairs, :4] == 0.0)
    cos = d_ab[self_pairs, 4]
    edgeless = np.array([graphs[g].count.size == 0 for g in a[self_pairs]])
    assert np.all(np.isnan(cos[edgeless])) and np.all(np.abs(cos[~edgeless]) < 1e-15)


def test_bad_indices_give_nan_and_leave_other_pairs_alone(cf, ctx, small):
    graphs, gs, a, b = small
    pa = np.array([0, -1, 5, len(graphs), 7], np.int32)
    pb = np.array([3, 2, 17, 1, -4], np.int32)
    got = cf.distances(ctx, gs, pa, pb).cpu().numpy()
    assert np.all(np.isnan(got[[1, 3, 4]]))
    check_distances(got[[0, 2]], graphs, pa[[0, 2]], pb[[0, 2]], 3.0)


def test_all_pairs_workload_sampled_and_deterministic(cf, ctx):
    cfg = config_graphs(1)
    graphs, pa, pb = cfg["graphs"], cfg["pair_a"], cfg["pair_b"]
    gs = cf.pack(ctx, graphs)
    got = cf.distances(ctx, gs, pa, pb).cpu().numpy()
    again = cf.distances(ctx, gs, pa, pb).cpu().numpy()
    np.testing.assert_array_equal(got, again)
    assert got.shape == (len(pa), 5) and np.all(np.isfinite(got))
    sizes = np.array([g.n for g in graphs])
    M = np.maximum(sizes[pa], sizes[pb])
    rng = np.random.default_rng(11)
    pick = np.unique(np.r_[rng.choice(len(pa), 64, replace=False), np.argmax(M), np.argmin(M)])
    check_distances(got[pick], graphs, pa[pick], pb[pick], 3.0)


def test_large_pairs_sampled(cf, ctx):
    cfg = config_graphs(2)
    graphs, pa, pb = cfg["graphs"], cfg["pair_a"], cfg["pair_b"]
    gs = cf.pack(ctx, graphs)
    got = cf.distances(ctx, gs, pa, pb).cpu().numpy()
    assert np.all(np.isfinite(got))
    sizes = np.array([g.n for g in graphs])
    M = np.maximum(sizes[pa], sizes[pb])
    pick = np.unique([int(np.argmax(M)), int(np.argmin(M)), 7])
    check_distances(got[pick], graphs, pa[pick], pb[pick], 3.0)
