"""Pins of the distance oracle (Table 1's elementwise measures, compared on
the pair's transition matrices scaled to a common size as Sections 4 and 4.1
describe) against what independent routines and the mathematics fix.  CPU
only."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.spatial.distance as ssd

import oracle
from cfgsynth import Grammar, make_cfg
from oracle import distances as dist

EUC, MAN, MIN, JAC, COS = range(5)


def _tm(n, seed, counts="trip"):
    g = make_cfg(n, Grammar(counts=counts), seed=seed)
    return oracle.transition_matrix(g.n, g.src, g.dst, g.count)


def _vectors(seed, n=257, zero_frac=0.4):
    rng = np.random.default_rng(seed)
    x = rng.random(n) * (rng.random(n) > zero_frac)
    y = rng.random(n) * (rng.random(n) > zero_frac)
    return x, y


def scipy_measures(x, y, p):
    """The same five measures from scipy's own routines; Jaccard from its
    Tanimoto form, which is the paper's ratio rewritten (numerator
    sum x^2 + sum y^2 - 2 sum x y)."""
    tanimoto = 1.0 - np.dot(x, y) / (np.dot(x, x) + np.dot(y, y) - np.dot(x, y))
    return np.array([ssd.euclidean(x, y), ssd.cityblock(x, y), ssd.minkowski(x, y, p), tanimoto,
                     ssd.cosine(x, y)])


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("p", [3.0, 1.5, 4.0])
def test_measures_match_scipy(seed, p):
    x, y = _vectors(seed)
    got = dist.elementwise_distances(x, y, p)
    np.testing.assert_allclose(got, scipy_measures(x, y, p), rtol=1e-12, atol=0)


@pytest.mark.parametrize("seed", range(5))
def test_jaccard_on_indicator_vectors_is_the_set_jaccard_distance(seed):
    rng = np.random.default_rng(100 + seed)
    xb, yb = rng.random(64) < 0.3, rng.random(64) < 0.5
    X, Y = set(np.flatnonzero(xb)), set(np.flatnonzero(yb))
    brute = len(X ^ Y) / len(X | Y)
    got = dist.elementwise_distances(xb.astype(float), yb.astype(float))[JAC]
    assert got == pytest.approx(brute, rel=1e-15)
    assert got == pytest.approx(ssd.jaccard(xb, yb), rel=1e-15)


def test_minkowski_orders_one_and_two_are_manhattan_and_euclidean():
    x, y = _vectors(7)
    d1 = dist.elementwise_distances(x, y, 1.0)
    d2 = dist.elementwise_distances(x, y, 2.0)
    assert d1[MIN] == pytest.approx(d1[MAN], rel=1e-14)
    assert d2[MIN] == pytest.approx(d2[EUC], rel=1e-14)


@pytest.mark.parametrize("x, y, want", [
    ([1.0, 0.0], [0.0, 1.0], [np.sqrt(2), 2.0, 2.0 ** (1 / 3), 1.0, 1.0]),
    ([1.0, 1.0], [2.0, 2.0], [np.sqrt(2), 2.0, 2.0 ** (1 / 3), 1 / 3, 0.0]),
    ([3.0, 4.0], [0.0, 0.0], [5.0, 7.0, 91.0 ** (1 / 3), 1.0, np.nan]),
    ([0.0, 0.0], [0.0, 0.0], [0.0, 0.0, 0.0, 0.0, np.nan]),
])
def test_hand_worked_vectors(x, y, want):
    np.testing.assert_allclose(dist.elementwise_distances(x, y, 3.0), want, rtol=1e-15, atol=1e-15)


def test_ranges_for_nonnegative_vectors():
    for seed in range(10):
        d = dist.elementwise_distances(*_vectors(seed))
        assert 0.0 <= d[JAC] <= 1.0 and 0.0 <= d[COS] <= 1.0
        assert d[EUC] <= d[MAN] and d[MIN] <= d[EUC] + 1e-15


def test_rejects_bad_order_and_lengths():
    x, y = _vectors(0)
    for p in (0.5, np.inf, np.nan):
        with pytest.raises(ValueError):
            dist.elementwise_distances(x, y, p)
    with pytest.raises(ValueError):
        dist.elementwise_distances(x, y[:-1])


def _corner_aligned_sample(X, M):
    """Order-1 sampling of X at p (m-1)/(M-1) along both axes through
    scipy.ndimage.map_coordinates (an independent bilinear routine)."""
    m = X.shape[0]
    t = np.arange(M) * (m - 1) / (M - 1)
    gi, gj = np.meshgrid(t, t, indexing="ij")
    return ndi.map_coordinates(X, [gi, gj], order=1, mode="nearest")


@pytest.mark.parametrize("m, M", [(5, 9), (8, 13), (12, 40), (3, 64)])
def test_pair_distances_compare_the_scaled_matrices(m, M):
    A, B = _tm(m, 3 * m), _tm(M, 5 * M)
    As = _corner_aligned_sample(A, M)
    want = scipy_measures(As.ravel(), B.ravel(), 3.0)
    np.testing.assert_allclose(oracle.pair_distances(A, B), want, rtol=1e-12, atol=1e-15)
    # Which graph is the smaller one does not matter.
    np.testing.assert_array_equal(oracle.pair_distances(B, A), oracle.pair_distances(A, B))


def test_equal_sizes_compare_the_matrices_unchanged():
    A, B = _tm(17, 1), _tm(17, 2)
    np.testing.assert_allclose(oracle.pair_distances(A, B), scipy_measures(A.ravel(), B.ravel(), 3.0),
                               rtol=1e-12, atol=0)


def test_a_graph_is_at_distance_zero_from_itself():
    A = _tm(23, 9)
    d = oracle.pair_distances(A, A)
    assert np.all(d[:JAC] == 0.0) and d[JAC] == 0.0
    assert abs(d[COS]) < 1e-15


def test_sparse_and_dense_inputs_agree():
    g1, g2 = make_cfg(90, seed=4), make_cfg(130, seed=6)
    Ad = oracle.transition_matrix(g1.n, g1.src, g1.dst, g1.count)
    Bd = oracle.transition_matrix(g2.n, g2.src, g2.dst, g2.count)
    As = oracle.transition_matrix_sparse(g1.n, g1.src, g1.dst, g1.count)
    Bs = oracle.transition_matrix_sparse(g2.n, g2.src, g2.dst, g2.count)
    np.testing.assert_allclose(oracle.pair_distances(As, Bs), oracle.pair_distances(Ad, Bd), rtol=1e-13, atol=1e-16)
