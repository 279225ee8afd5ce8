"""Pins of the damped IsoRank oracle (Table 1, row "Iso", full form
(I - alpha Q x P) x = (1 - alpha) E) against what the mathematics fixes: a
dense linear solve with the explicit Kronecker operator, IsoRank's own
matrix built entry by entry from neighbour counts, the contraction bound,
special cases and invariants; plus planted mistakes that each fail a pin.
CPU only."""
import numpy as np
import pytest

import oracle
from cfgsynth import Grammar, make_cfg
from oracle import damped as dp


def _tm(n, seed, counts="trip"):
    g = make_cfg(n, Grammar(counts=counts), seed=seed)
    return oracle.transition_matrix(g.n, g.src, g.dst, g.count)


def _random_digraph(n, seed, density=0.35):
    """Non-negative matrix with some empty rows and columns."""
    rng = np.random.default_rng(seed)
    X = rng.random((n, n)) * (rng.random((n, n)) < density)
    X[rng.integers(n)] = 0.0
    X[:, rng.integers(n)] = 0.0
    return X


def explicit_solution(A, B, alpha, E):
    """x* of (I - alpha M_hat) x = (1 - alpha) E with M = kron(B, A) +
    kron(B^T, A^T) written out and its columns divided by their sums."""
    M = np.kron(B, A) + np.kron(B.T, A.T)
    d = M.sum(axis=0)
    Mh = np.zeros_like(M)
    Mh[:, d > 0] = M[:, d > 0] / d[d > 0]
    n = M.shape[0]
    x = np.linalg.solve(np.eye(n) - alpha * Mh, (1.0 - alpha) * E.ravel())
    return x.reshape(E.shape)


def _pairs():
    yield _tm(7, 1), _tm(5, 2)
    yield _tm(9, 3, "uniform"), _tm(9, 4)
    yield _random_digraph(6, 5), _random_digraph(4, 6)
    yield _random_digraph(5, 7), _tm(8, 8)


@pytest.mark.parametrize("alpha", [0.2, 0.5, 0.85, 0.95])
@pytest.mark.parametrize("k", range(4))
def test_iteration_reaches_the_dense_solve_within_its_bound(alpha, k):
    A, B = list(_pairs())[k]
    nA, nB = A.shape[0], B.shape[0]
    E = np.full((nB, nA), 1.0 / (nA * nB))
    xs = explicit_solution(A, B, alpha, E)
    S, nu, delta, iters, status, its = dp.damped_iteration(A, B, alpha, None, max_iter=3000, tol=1e-14,
                                                            keep_iterates=True)
    x = its[-1]
    assert status == oracle.CONVERGED
    assert np.abs(x - xs).sum() <= alpha * delta / (1 - alpha) + 1e-13
    np.testing.assert_allclose(S, xs / np.linalg.norm(xs), rtol=0, atol=1e-12)
    assert nu == pytest.approx(np.linalg.norm(xs), rel=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_user_prior_matches_the_dense_solve(seed):
    A, B = _tm(6, 10 + seed), _tm(7, 20 + seed)
    rng = np.random.default_rng(seed)
    P = rng.random((7, 6)) * (rng.random((7, 6)) < 0.6)
    P[0, 0] = 1.0
    E = P / P.sum()
    xs = explicit_solution(A, B, 0.7, E)
    S = dp.damped_iteration(A, B, 0.7, P * 3.0, max_iter=2000, tol=1e-15)[0]
    np.testing.assert_allclose(S, xs / np.linalg.norm(xs), rtol=0, atol=1e-12)


@pytest.mark.parametrize("k", range(4))
def test_column_sums_are_those_of_the_explicit_kronecker_operator(k):
    A, B = list(_pairs())[k]
    M = np.kron(B, A) + np.kron(B.T, A.T)
    np.testing.assert_allclose(dp.column_sums(A, B).ravel(), M.sum(axis=0), rtol=1e-14, atol=0)


def _undirected(n, seed):
    rng = np.random.default_rng(seed)
    X = np.triu((rng.random((n, n)) < 0.5).astype(float), 1)
    X = X + X.T
    for v in range(n):  # no isolated node
        if X[v].sum() == 0:
            u = (v + 1) % n
            X[v, u] = X[u, v] = 1.0
    return X


@pytest.mark.parametrize("seed", range(4))
def test_undirected_graphs_give_isorank_matrix_from_neighbour_counts(seed):
    A, B = _undirected(5, seed), _undirected(4, 40 + seed)
    nA, nB = 5, 4
    # IsoRank: entry ((i, j), (u, v)) = 1 / (|N(u)| |N(v)|) when u ~ i in B and v ~ j in A
    iso = np.zeros((nB * nA, nB * nA))
    for i in range(nB):
        for j in range(nA):
            for u in range(nB):
                for v in range(nA):
                    if B[i, u] and A[j, v]:
                        iso[i * nA + j, u * nA + v] = 1.0 / (B[u].sum() * A[v].sum())
    got = np.zeros_like(iso)
    for c in range(nB * nA):
        X = np.zeros((nB, nA))
        X.flat[c] = 1.0
        got[:, c] = dp.apply_normalised(A, B, X).ravel()
    np.testing.assert_allclose(got, iso, rtol=1e-15, atol=0)


def test_alpha_zero_returns_the_prior():
    A, B = _tm(6, 1), _tm(9, 2)
    rng = np.random.default_rng(3)
    P = rng.random((9, 6))
    S, nu, delta, iters, status = dp.damped_iteration(A, B, 0.0, P)
    E = P / P.sum()
    np.testing.assert_allclose(S, E / np.linalg.norm(E), rtol=1e-15)
    assert (iters, status, delta) == (1, oracle.CONVERGED, 0.0)


def test_mass_is_kept_when_no_column_of_the_operator_is_zero():
    # cycles with a chord: every node has in- and out-edges, so d > 0 everywhere
    def cyc(n, seed):
        rng = np.random.default_rng(seed)
        X = np.zeros((n, n))
        for v in range(n):
            X[v, (v + 1) % n] = rng.integers(1, 100)
        X[0, n // 2] = 7.0
        return X / X.sum(axis=1, keepdims=True)
    A, B = cyc(6, 1), cyc(5, 2)
    assert (dp.column_sums(A, B) > 0).all()
    its = dp.damped_iteration(A, B, 0.9, None, max_iter=40, tol=0.0, keep_iterates=True)[-1]
    for x in its:
        assert x.sum() == pytest.approx(1.0, abs=1e-14)


def test_steps_contract_by_alpha():
    A, B = _tm(12, 5), _tm(10, 6)
    for alpha in (0.3, 0.8, 0.97):
        its = dp.damped_iteration(A, B, alpha, None, max_iter=60, tol=0.0, keep_iterates=True)[-1]
        steps = [np.abs(its[k] - its[k - 1]).sum() for k in range(1, len(its))]
        for a, b in zip(steps, steps[1:]):
            assert b <= alpha * a * (1 + 1e-12) + 1e-17


def test_swap_transposes_and_permutation_relabels():
    A, B = _tm(8, 11), _tm(6, 12)
    S = dp.damped_iteration(A, B, 0.8, None, 400, 1e-15)[0]
    St = dp.damped_iteration(B, A, 0.8, None, 400, 1e-15)[0]
    np.testing.assert_allclose(St, S.T, rtol=0, atol=1e-14)
    rng = np.random.default_rng(0)
    pa, pb = rng.permutation(8), rng.permutation(6)
    PA, PB = np.eye(8)[pa], np.eye(6)[pb]
    Sp = dp.damped_iteration(PA @ A @ PA.T, PB @ B @ PB.T, 0.8, None, 400, 1e-15)[0]
    np.testing.assert_allclose(Sp, PB @ S @ PA.T, rtol=0, atol=1e-14)


def test_power_of_two_scaling_is_bit_exact():
    A, B = _tm(9, 21), _tm(7, 22)
    S = dp.damped_iteration(A, B, 0.85)[0]
    assert np.array_equal(dp.damped_iteration(4.0 * A, B, 0.85)[0], S)
    assert np.array_equal(dp.damped_iteration(A, 0.5 * B, 0.85)[0], S)


def test_score_is_the_greedy_sum_on_the_returned_s():
    A, B = _tm(10, 31), _tm(13, 32)
    r = dp.score_pair_damped(A, B, 0.85)
    m, sc = oracle.greedy_match(r.S)
    assert np.array_equal(m, r.match) and sc == r.score
    assert np.linalg.norm(r.S) == pytest.approx(1.0, rel=1e-15)


def test_bad_arguments_are_refused():
    A, B = _tm(5, 1), _tm(5, 2)
    for alpha in (-0.1, 1.0, np.nan):
        with pytest.raises(ValueError):
            dp.damped_iteration(A, B, alpha)
    with pytest.raises(ValueError):
        dp.damped_iteration(A, B, 0.5, -np.ones((5, 5)))
    with pytest.raises(ValueError):
        dp.damped_iteration(A, B, 0.5, np.zeros((5, 5)))


# ---------------------------------------------------------------- planted mistakes
def _dense_pin_holds(alpha=0.85):
    A, B = _tm(7, 1), _tm(5, 2)
    E = np.full((5, 7), 1.0 / 35)
    xs = explicit_solution(A, B, alpha, E)
    S = dp.damped_iteration(A, B, alpha, None, 2000, 1e-15)[0]
    return np.allclose(S, xs / np.linalg.norm(xs), rtol=0, atol=1e-10)


def test_unmutated_damped_oracle_passes():
    assert _dense_pin_holds()


MUTANTS = {
    "row sums in both terms of d": ("column_sums",
                                    lambda A, B: 2.0 * np.outer(np.asarray(B).sum(1), np.asarray(A).sum(1))),
    "only the direct term in d": ("column_sums",
                                  lambda A, B: np.outer(np.asarray(B).sum(0), np.asarray(A).sum(0))),
    "dropped transpose term": ("apply_operator", lambda A, B, S: B @ S @ A.T),
    "transposed A": ("apply_operator", lambda A, B, S: B @ S @ A + B.T @ S @ A.T),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_damped_mutants_fail_the_dense_pin(monkeypatch, name):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(dp, attr, fn)
    assert not _dense_pin_holds()


def test_mutant_without_the_damping_factor_on_the_prior_fails(monkeypatch):
    real = dp.prior_of
    monkeypatch.setattr(dp, "prior_of", lambda nA, nB, prior=None: real(nA, nB, prior) / 0.15)
    # S is scale-free, so the planted factor shows in the un-normalised norm
    A, B = _tm(7, 1), _tm(5, 2)
    xs = explicit_solution(A, B, 0.85, np.full((5, 7), 1.0 / 35))
    nu = dp.damped_iteration(A, B, 0.85, None, 2000, 1e-15)[1]
    assert nu != pytest.approx(np.linalg.norm(xs), rel=1e-6)
