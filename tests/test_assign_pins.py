"""Pins of the optimal-assignment oracle (the matching of min(n_A, n_B) node
pairs with the largest total similarity) against scipy's linear assignment
solver, brute force over all matchings on tiny matrices, and properties of
the optimum; plus planted mistakes that fail a pin.  CPU only."""
import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle
from cfgsynth import Grammar, make_cfg
from oracle import assign as asg


def _total(S, match):
    return sum(S[i, j] for i, j in enumerate(match) if j >= 0)


def _valid(match, nB, nA):
    cols = [j for j in match if j >= 0]
    assert len(cols) == min(nB, nA) and len(set(cols)) == len(cols)
    assert all(0 <= j < nA for j in cols)


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (7, 1), (5, 5), (6, 9), (9, 6), (40, 40), (33, 70), (70, 33)])
@pytest.mark.parametrize("seed", range(3))
def test_total_equals_scipy_linear_sum_assignment(shape, seed):
    rng = np.random.default_rng(seed)
    S = rng.random(shape)
    match, score = asg.optimal_assignment(S)
    _valid(match, *shape)
    r, c = linear_sum_assignment(S, maximize=True)
    assert score == pytest.approx(S[r, c].sum(), rel=1e-13, abs=1e-15)
    assert score == pytest.approx(_total(S, match), rel=1e-15)


def _brute(S):
    nB, nA = S.shape
    best, arg = -np.inf, None
    if nB <= nA:
        for cols in itertools.permutations(range(nA), nB):
            t = sum(S[i, c] for i, c in enumerate(cols))
            if t > best:
                best, arg = t, list(cols)
    else:
        for rows in itertools.permutations(range(nB), nA):
            t = sum(S[r, j] for j, r in enumerate(rows))
            if t > best:
                best = t
                arg = [-1] * nB
                for j, r in enumerate(rows):
                    arg[r] = j
    return np.array(arg), best


@pytest.mark.parametrize("shape", [(2, 2), (3, 4), (4, 3), (5, 5), (4, 6), (6, 4), (6, 6)])
@pytest.mark.parametrize("seed", range(4))
def test_brute_force_on_tiny_matrices(shape, seed):
    S = np.random.default_rng(10 + seed).random(shape)   # distinct values: one optimum
    match, score = asg.optimal_assignment(S)
    bm, bt = _brute(S)
    assert np.array_equal(match, bm)
    assert score == pytest.approx(bt, rel=1e-14)


def test_similarity_matrices_of_cfg_pairs():
    for seed in range(3):
        ga = make_cfg(20 + 7 * seed, Grammar(counts="trip"), seed=seed)
        gb = make_cfg(15 + 11 * seed, Grammar(counts="trip"), seed=seed + 100)
        A = oracle.transition_matrix(ga.n, ga.src, ga.dst, ga.count)
        B = oracle.transition_matrix(gb.n, gb.src, gb.dst, gb.count)
        S = oracle.score_pair(A, B).S
        match, score = asg.optimal_assignment(S)
        _valid(match, *S.shape)
        r, c = linear_sum_assignment(S, maximize=True)
        assert score == pytest.approx(S[r, c].sum(), rel=1e-13)
        gm, gscore = oracle.greedy_match(S)
        # the greedy matching is maximal, so it keeps at least half the optimum
        assert gscore <= score * (1 + 1e-15) and gscore >= 0.5 * score


def test_ties_are_broken_the_same_way_every_time_and_stay_optimal():
    S = np.ones((6, 8))
    S[2, :] = 2.0
    S[:, 5] = 3.0
    m1, s1 = asg.optimal_assignment(S)
    m2, s2 = asg.optimal_assignment(S.copy())
    assert np.array_equal(m1, m2) and s1 == s2
    _valid(m1, 6, 8)
    r, c = linear_sum_assignment(S, maximize=True)
    assert s1 == pytest.approx(S[r, c].sum(), rel=1e-15)


def test_row_shift_and_permutations():
    rng = np.random.default_rng(4)
    S = rng.random((12, 12))
    m, sc = asg.optimal_assignment(S)
    # adding a constant to one row changes every full matching's total equally
    S2 = S.copy()
    S2[3] += 5.0
    m2, sc2 = asg.optimal_assignment(S2)
    assert np.array_equal(m2, m) and sc2 == pytest.approx(sc + 5.0, rel=1e-14)
    pr, pc = rng.permutation(12), rng.permutation(12)
    mp, scp = asg.optimal_assignment(S[np.ix_(pr, pc)])
    assert scp == pytest.approx(sc, rel=1e-14)
    for i in range(12):   # row pr[i] of S is matched to column pc[mp[i]]
        assert m[pr[i]] == pc[mp[i]]


def test_non_finite_input_is_refused():
    S = np.ones((3, 3))
    S[1, 1] = np.nan
    with pytest.raises(ValueError):
        asg.optimal_assignment(S)


# ---------------------------------------------------------------- planted mistakes
def _pin_holds(fn):
    rng = np.random.default_rng(99)
    for shape in [(6, 9), (9, 6), (12, 12)]:
        S = rng.random(shape)
        match, score = fn(S)
        r, c = linear_sum_assignment(S, maximize=True)
        if abs(score - S[r, c].sum()) > 1e-12:
            return False
    return True


def _greedy_as_assignment(S):
    return oracle.greedy_match(S)


def _no_potential_shift(S):
    """Mutant: the tree's slack is not subtracted from the unused columns."""
    S = np.asarray(S, np.float64)
    nB, nA = S.shape
    transpose = nB > nA
    C = -(S.T if transpose else S)
    n, m = C.shape
    u, v = np.zeros(n + 1), np.zeros(m + 1)
    p, way = np.zeros(m + 1, np.int64), np.zeros(m + 1, np.int64)
    for i in range(1, n + 1):
        p[0], j0 = i, 0
        minv, used = np.full(m + 1, np.inf), np.zeros(m + 1, bool)
        while True:
            used[j0] = True
            i0 = p[j0]
            free = ~used[1:]
            cur = C[i0 - 1] - u[i0] - v[1:]
            better = free & (cur < minv[1:])
            minv[1:][better] = cur[better]
            way[1:][better] = j0
            cand = np.where(free, minv[1:], np.inf)
            j1 = int(np.argmin(cand)) + 1
            delta = cand[j1 - 1]
            u[p[used]] += delta
            v[used] -= delta
            j0 = j1
            if p[j0] == 0:
                break
        while j0 != 0:
            j1 = way[j0]
            p[j0] = p[j1]
            j0 = j1
    match = np.full(nB, -1)
    for j in range(1, m + 1):
        if p[j]:
            if transpose:
                match[j - 1] = p[j] - 1
            else:
                match[p[j] - 1] = j - 1
    return match, _total(S, match)


def test_unmutated_oracle_passes():
    assert _pin_holds(asg.optimal_assignment)


@pytest.mark.parametrize("fn", [_greedy_as_assignment, _no_potential_shift])
def test_mutants_fail_the_scipy_pin(fn):
    assert not _pin_holds(fn)
