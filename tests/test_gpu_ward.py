"""Parity of Ward's clustering (cfsim_ward, Section 6.2) with the FP64
oracle.  Both take the squared Euclidean distances in feature order and the
Lance-Williams recurrence in the same order without fused operations, under
the same tie rule, so the linkage must be identical bit for bit (merged
clusters, heights, sizes) on inputs the oracle finishes quickly; larger
inputs are checked against scipy's Ward linkage (merges identical on inputs
without ties, heights equal to scipy's squared to 1e-12 relative)."""
import numpy as np
import pytest
from scipy.cluster.hierarchy import linkage

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


@pytest.mark.parametrize("n,f", [(2, 1), (3, 2), (17, 3), (64, 5), (65, 33), (130, 40)])
def test_linkage_equals_the_oracle_bit_for_bit(cf, ctx, n, f):
    X = np.random.default_rng(n * 100 + f).random((n, f))
    Z = cf.ward(ctx, X).cpu().numpy()
    np.testing.assert_array_equal(Z, oracle.ward_linkage(X))


def test_ties_and_duplicates(cf, ctx):
    rng = np.random.default_rng(3)
    X = rng.integers(0, 3, size=(40, 2)).astype(np.float64)   # many equal distances and duplicate points
    Z = cf.ward(ctx, X).cpu().numpy()
    np.testing.assert_array_equal(Z, oracle.ward_linkage(X))
    X = np.ones((6, 3))
    np.testing.assert_array_equal(cf.ward(ctx, X).cpu().numpy(), oracle.ward_linkage(X))


def test_single_observation_and_non_finite(cf, ctx):
    assert cf.ward(ctx, np.ones((1, 4))).shape == (0, 4)
    X = np.random.default_rng(4).random((9, 3))
    X[4, 1] = np.nan
    assert np.isnan(cf.ward(ctx, X).cpu().numpy()).all()


@pytest.mark.parametrize("n,f", [(600, 16), (2048, 8)])
def test_large_inputs_against_scipy(cf, ctx, n, f):
    X = np.random.default_rng(n).random((n, f))
    Z = cf.ward(ctx, X).cpu().numpy()
    R = linkage(X, method="ward")
    np.testing.assert_array_equal(Z[:, [0, 1, 3]], R[:, [0, 1, 3]])
    np.testing.assert_allclose(Z[:, 2], R[:, 2] ** 2, rtol=1e-12, atol=1e-14)


def test_clustering_of_the_score_matrix(cf, ctx):
    """Feature vector of a graph = its row of the all-pairs score matrix
    (FP64 batched path, self pairs on the diagonal)."""
    w = config_graphs(1, scale=48 / 256)
    G = len(w["graphs"])
    gs = cf.pack(ctx, w["graphs"])
    ia, ib = np.triu_indices(G)
    res, _, _ = cf.score_batch(ctx, gs, ia.astype(np.int32), ib.astype(np.int32), dtype="f64", want_match=False)
    M = np.zeros((G, G))
    M[ia, ib] = res["score"]
    M[ib, ia] = res["score"]
    Z = cf.ward(ctx, M).cpu().numpy()
    np.testing.assert_array_equal(Z, oracle.ward_linkage(M))
