"""Pins of the Ward clustering oracle (Section 6.2: Ward's minimum variance
method from squared Euclidean distances) against scipy's Ward linkage, the
variance-increase definition recomputed from the clusters' members, brute
force over every candidate merge, and monotone heights; plus planted
mistakes.  CPU only."""
import numpy as np
import pytest
from scipy.cluster.hierarchy import fcluster, linkage

from oracle import ward as wd


def _members(Z, n):
    groups = {i: [i] for i in range(n)}
    out = []
    for s, (a, b, h, c) in enumerate(Z):
        g = groups.pop(int(a)) + groups.pop(int(b))
        groups[n + s] = g
        out.append(g)
    return out


@pytest.mark.parametrize("n,f", [(2, 1), (3, 2), (10, 3), (40, 5), (97, 8), (150, 20)])
@pytest.mark.parametrize("seed", range(3))
def test_equals_scipy_ward_linkage(n, f, seed):
    X = np.random.default_rng(seed).random((n, f))
    Z = wd.ward_linkage(X)
    R = linkage(X, method="ward")
    np.testing.assert_array_equal(Z[:, [0, 1, 3]], R[:, [0, 1, 3]])
    # scipy's heights are the square roots of the squared-distance form
    np.testing.assert_allclose(Z[:, 2], R[:, 2] ** 2, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_heights_are_twice_the_variance_increase_of_the_members(seed):
    rng = np.random.default_rng(10 + seed)
    X = rng.normal(size=(30, 4))
    Z = wd.ward_linkage(X)
    n = len(X)
    groups = {i: [i] for i in range(n)}
    for s, (a, b, h, c) in enumerate(Z):
        A, B = groups.pop(int(a)), groups.pop(int(b))
        ca, cb = X[A].mean(axis=0), X[B].mean(axis=0)
        inc = len(A) * len(B) / (len(A) + len(B)) * np.sum((ca - cb) ** 2)
        # equally, the rise of the within-cluster sum of squares
        ess = lambda G: np.sum((X[G] - X[G].mean(axis=0)) ** 2)
        assert inc == pytest.approx(ess(A + B) - ess(A) - ess(B), rel=1e-9, abs=1e-12)
        assert h == pytest.approx(2 * inc, rel=1e-11)
        # brute force: no other pair of current clusters merges more cheaply
        cur = list(groups.values())
        for x in range(len(cur)):
            for y in range(x + 1, len(cur)):
                P, Q = cur[x], cur[y]
                other = len(P) * len(Q) / (len(P) + len(Q)) * np.sum((X[P].mean(0) - X[Q].mean(0)) ** 2)
                assert 2 * other >= h * (1 - 1e-9)
        groups[n + s] = A + B
        assert c == len(A) + len(B)


def test_heights_never_decrease_and_flat_clusters_match_scipy():
    X = np.random.default_rng(5).random((120, 6))
    Z = wd.ward_linkage(X)
    assert np.all(np.diff(Z[:, 2]) >= 0)
    R = linkage(X, method="ward")
    for k in (2, 5, 12):
        a = fcluster(np.column_stack([Z[:, :2], np.sqrt(Z[:, 2]), Z[:, 3]]), k, "maxclust")
        b = fcluster(R, k, "maxclust")
        assert np.array_equal(a, b)


def test_ties_take_the_smallest_pair_and_single_observation():
    X = np.array([[0.0], [1.0], [2.0], [3.0]])   # equal gaps: (0, 1) first
    Z = wd.ward_linkage(X)
    assert list(Z[0, :2]) == [0, 1] and Z[0, 2] == 1.0
    assert wd.ward_linkage(np.zeros((1, 3))).shape == (0, 4)
    # identical points merge at height 0
    Z = wd.ward_linkage(np.ones((5, 2)))
    assert np.all(Z[:, 2] == 0.0)


def test_squared_distances_are_the_definition():
    X = np.random.default_rng(8).random((9, 5))
    D = wd.squared_distances(X)
    for i in range(9):
        for j in range(9):
            assert D[i, j] == pytest.approx(np.sum((X[i] - X[j]) ** 2), rel=1e-15, abs=1e-300)


# ---------------------------------------------------------------- planted mistakes
def _pin_holds():
    X = np.random.default_rng(3).random((40, 5))
    Z = wd.ward_linkage(X)
    R = linkage(X, method="ward")
    return np.array_equal(Z[:, [0, 1, 3]], R[:, [0, 1, 3]]) and np.allclose(Z[:, 2], R[:, 2] ** 2, rtol=1e-12)


MUTANTS = {
    "average linkage update": lambda dki, dkj, dij, ni, nj, nk: (ni * dki + nj * dkj) / (ni + nj),
    "dropped -n_k d_ij term": lambda dki, dkj, dij, ni, nj, nk: ((ni + nk) * dki + (nj + nk) * dkj) / (ni + nj + nk),
    "unweighted": lambda dki, dkj, dij, ni, nj, nk: (dki + dkj - dij / 2) / 2,
}


def test_unmutated_oracle_passes():
    assert _pin_holds()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants_fail_the_scipy_pin(monkeypatch, name):
    monkeypatch.setattr(wd, "ward_update", MUTANTS[name])
    assert not _pin_holds()


def test_mutant_unsquared_distances_fails(monkeypatch):
    real = wd.squared_distances
    monkeypatch.setattr(wd, "squared_distances", lambda X: np.sqrt(real(X)))
    assert not _pin_holds()
