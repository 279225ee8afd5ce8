"""Plant plausible mistakes in the oracle (CPU only) and check that the pins
reject every one of them.  Nothing here touches a GPU."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from cfgsynth import Grammar, make_cfg
from oracle import cfsim_ref as ref
from tests.golden.fixtures import pathfinder_fig3


def _pair(seed=0):
    ga = make_cfg(8, Grammar(counts="trip"), seed=seed)
    gb = make_cfg(6, Grammar(counts="trip"), seed=seed + 50)
    A = oracle.transition_matrix(ga.n, ga.src, ga.dst, ga.count)
    B = oracle.transition_matrix(gb.n, gb.src, gb.dst, gb.count)
    return A, B, ga, gb


def _closed_form_holds(A, B, K=25):
    M = np.kron(B, A) + np.kron(B.T, A.T)
    lam, V = np.linalg.eigh(M)
    s0 = np.full(M.shape[0], 1 / np.sqrt(M.shape[0]))
    x = V @ (((lam / np.abs(lam).max()) ** K) * (V.T @ s0))
    x /= np.linalg.norm(x)
    S = oracle.coupled_iteration(A, B, K, -1.0)[0]
    return np.allclose(S.ravel(), x, atol=1e-10)


MUTANT_OPERATORS = {
    "dropped transpose term": lambda A, B, S: B @ S @ A.T,
    "dropped direct term": lambda A, B, S: B.T @ S @ A,
    "transposed A": lambda A, B, S: B @ S @ A + B.T @ S @ A.T,
    "transposed B": lambda A, B, S: B.T @ S @ A.T + B @ S @ A,
    "wrong sign": lambda A, B, S: B @ S @ A.T - B.T @ S @ A,
    "extra identity": lambda A, B, S: B @ S @ A.T + B.T @ S @ A + S,
}


def test_unmutated_oracle_passes():
    A, B, *_ = _pair()
    assert _closed_form_holds(A, B)


@pytest.mark.parametrize("name", sorted(MUTANT_OPERATORS))
def test_operator_mutants_fail_the_eigen_pin(monkeypatch, name):
    A, B, *_ = _pair()
    monkeypatch.setattr(ref, "apply_operator", MUTANT_OPERATORS[name])
    assert not _closed_form_holds(A, B)


def test_mutant_update_count_fails_the_eigen_pin(monkeypatch):
    A, B, *_ = _pair()
    real = ref.coupled_iteration

    def one_extra(A, B, max_iter=200, tol=1e-12, keep_iterates=False):
        return real(A, B, max_iter + 1, tol, keep_iterates)
    monkeypatch.setattr(oracle, "coupled_iteration", one_extra)
    assert not _closed_form_holds(A, B)


def _naive_greedy(S):
    """The pin: repeatedly the largest free entry, ties to the smaller flat
    index, by a plain double loop (no sorting)."""
    S = np.asarray(S, np.float64)
    nB, nA = S.shape
    rows, cols = set(range(nB)), set(range(nA))
    match = np.full(nB, -1)
    while rows and cols:
        best = None
        for i in sorted(rows):
            for j in sorted(cols):
                if best is None or S[i, j] > S[best]:
                    best = (i, j)
        match[best[0]] = best[1]
        rows.discard(best[0])
        cols.discard(best[1])
    return match


def _greedy_pin_holds(cases):
    return all(np.array_equal(ref.greedy_match(S)[0], _naive_greedy(S)) for S in cases)


def test_mutant_tie_break_fails_the_naive_greedy_pin(monkeypatch):
    """A reversed tie-break planted into the oracle's greedy fails the pin."""
    rng = np.random.default_rng(4)
    cases = [np.array([[1.0, 1.0], [1.0, 0.0]]), np.round(rng.random((5, 4)), 1), np.ones((3, 3))]
    assert _greedy_pin_holds(cases)

    def reversed_ties(S):
        nB, nA = S.shape
        flat = np.asarray(S, np.float64).ravel()
        order = np.lexsort((-np.arange(flat.size), -flat))
        used_r, used_c, match = set(), set(), np.full(nB, -1, np.int32)
        for idx in order:
            i, j = divmod(int(idx), nA)
            if i not in used_r and j not in used_c:
                match[i] = j
                used_r.add(i)
                used_c.add(j)
        return match, 0.0
    monkeypatch.setattr(ref, "greedy_match", reversed_ties)
    assert not _greedy_pin_holds(cases)


def test_mutant_backward_fails_finite_differences(monkeypatch):
    A, B, ga, gb = _pair(3)
    K = 20
    r = oracle.score_pair(A, B, K, -1.0)

    def fd(e):
        p, q = int(ga.src[e]), int(ga.dst[e])
        f = []
        for h in (1e-6, -1e-6):
            X = A.copy()
            X[p, q] += h
            S = oracle.coupled_iteration(X, B, K, -1.0)[0]
            f.append(sum(S[i, j] for i, j in enumerate(r.match) if j >= 0))
        return (f[0] - f[1]) / 2e-6

    dA, _ = oracle.backward(A, B, K, r.match)
    good = all(abs(fd(e) - dA[ga.src[e], ga.dst[e]]) < 1e-8 for e in range(ga.nnz))
    assert good
    # mutant: forget the projection term of the normalisation adjoint
    orig = ref.backward

    def no_projection(A_, B_, iters, match):
        A_ = np.asarray(A_)
        B_ = np.asarray(B_)
        S, nu, d, k, st, its, nus = ref.coupled_iteration(A_, B_, iters, -1.0, keep_iterates=True)
        G = np.zeros_like(S)
        for i, j in enumerate(match):
            if j >= 0:
                G[i, j] = 1
        dA_ = np.zeros_like(A_)
        for kk in range(k - 1, -1, -1):
            Yb = G / nus[kk]
            dA_ += Yb.T @ B_ @ its[kk] + its[kk].T @ B_ @ Yb
            G = B_.T @ Yb @ A_ + B_ @ Yb @ A_.T
        return dA_, None
    dA_bad, _ = no_projection(A, B, K, r.match)
    assert not all(abs(fd(e) - dA_bad[ga.src[e], ga.dst[e]]) < 1e-8 for e in range(ga.nnz))
    assert orig is ref.backward


def test_mutant_resize_grid_fails_zoom_pin():
    X = np.random.default_rng(2).random((5, 5))
    Z = ndi.zoom(X, 9 / 5, order=1, grid_mode=False, mode="nearest")
    good = oracle.resize_bilinear(X, 9)
    assert np.allclose(good, Z, atol=1e-15)
    # mutant: half-pixel-centred grid (grid_mode=True sampling)
    from scipy.interpolate import RegularGridInterpolator
    t = (np.arange(9) + 0.5) * 5 / 9 - 0.5
    t = np.clip(t, 0, 4)
    f = RegularGridInterpolator((np.arange(5), np.arange(5)), X)
    P, Q = np.meshgrid(t, t, indexing="ij")
    bad = f(np.stack([P.ravel(), Q.ravel()], axis=1)).reshape(9, 9)
    assert not np.allclose(bad, Z, atol=1e-6)


def test_pathfinder_fixture_invariants_both_modes():
    """Figure 3 matrices as inputs (no printed output: parity unpinned)."""
    m = pathfinder_fig3()
    K, Mx = m["kepler"], m["maxwell"]
    assert K.shape == (6, 6) and Mx.shape == (4, 4)
    for mode in ("none", "bilinear"):
        r = oracle.score_pair(Mx, K, resize=mode)
        assert abs(np.linalg.norm(r.S) - 1) < 1e-14 and (r.S >= 0).all()
        r2 = oracle.score_pair(K, Mx, resize=mode)
        np.testing.assert_allclose(r2.S, r.S.T, atol=1e-13)
        if mode == "bilinear":
            assert r.S.shape == (6, 6)
        else:
            assert r.S.shape == (6, 4)


# ---------------------------------------------------------------- distances
def _distance_pins_hold(fn) -> bool:
    """The scipy, set-Jaccard and scaled-pair pins of tests/test_distance_pins.py
    applied to `fn` in place of the oracle's elementwise_distances."""
    from tests.test_distance_pins import _corner_aligned_sample, _tm, _vectors, scipy_measures
    ok = True
    for seed in range(3):
        x, y = _vectors(seed)
        ok &= np.allclose(fn(x, y, 3.0), scipy_measures(x, y, 3.0), rtol=1e-12, atol=0)
    rng = np.random.default_rng(1)
    xb, yb = rng.random(64) < 0.3, rng.random(64) < 0.5
    X, Y = set(np.flatnonzero(xb)), set(np.flatnonzero(yb))
    ok &= np.isclose(fn(xb.astype(float), yb.astype(float), 3.0)[3], len(X ^ Y) / len(X | Y), rtol=1e-15)
    A, B = _tm(5, 15), _tm(9, 45)
    As = _corner_aligned_sample(A, 9)
    ok &= np.allclose(fn(*oracle.scaled_pair(A, B), 3.0), scipy_measures(As.ravel(), B.ravel(), 3.0),
                      rtol=1e-12, atol=1e-15)
    return bool(ok)


def _with_sums(transform):
    def fn(x, y, p=3.0):
        x = np.asarray(x, float).ravel()
        y = np.asarray(y, float).ravel()
        return transform(x, y, p)
    return fn


MUTANT_DISTANCES = {
    "euclidean without the root": _with_sums(
        lambda x, y, p: np.r_[np.sum((x - y) ** 2), oracle.elementwise_distances(x, y, p)[1:]]),
    "manhattan of squares": _with_sums(
        lambda x, y, p: np.r_[oracle.elementwise_distances(x, y, p)[:1], np.sum((x - y) ** 2),
                              oracle.elementwise_distances(x, y, p)[2:]]),
    "minkowski without the root": _with_sums(
        lambda x, y, p: np.r_[oracle.elementwise_distances(x, y, p)[:2], np.sum(np.abs(x - y) ** p),
                              oracle.elementwise_distances(x, y, p)[3:]]),
    "jaccard denominator adds the cross term": _with_sums(
        lambda x, y, p: np.r_[oracle.elementwise_distances(x, y, p)[:3],
                              np.sum((x - y) ** 2) / (x @ x + y @ y + x @ y),
                              oracle.elementwise_distances(x, y, p)[4:]]),
    "cosine without the square roots": _with_sums(
        lambda x, y, p: np.r_[oracle.elementwise_distances(x, y, p)[:4], 1 - (x @ y) / ((x @ x) * (y @ y))]),
}


def test_unmutated_distances_pass():
    assert _distance_pins_hold(oracle.elementwise_distances)


@pytest.mark.parametrize("name", sorted(MUTANT_DISTANCES))
def test_distance_mutants_fail_the_pins(name):
    assert not _distance_pins_hold(MUTANT_DISTANCES[name])


def test_unscaled_pair_fails_the_scaled_pin():
    from tests.test_distance_pins import _corner_aligned_sample, _tm, scipy_measures
    A, B = _tm(5, 15), _tm(9, 45)
    # A mutant that scales by nearest-node repetition instead of the order-1 spline.
    idx = np.rint(np.arange(9) * 4 / 8).astype(int)
    x = A[np.ix_(idx, idx)].ravel()
    want = scipy_measures(_corner_aligned_sample(A, 9).ravel(), B.ravel(), 3.0)
    assert not np.allclose(oracle.elementwise_distances(x, B.ravel(), 3.0), want, rtol=1e-12)
