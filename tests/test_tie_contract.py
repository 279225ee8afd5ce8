"""Pins of the matching contract used by the GPU parity tests (CPU only).

Every S of the method is non-negative, so the GPU's rounding errors are
relative per entry.  The contract: if every entry of S' is within a relative
eps of S, and the relative greedy margin m of S (`relative_margin`: the
smallest 1 - q / v over greedy picks v and their rivals q, entries of the
pick's row or column whose other line was still free at the pick) exceeds
2 eps, then S' has the same greedy matching as S.  These tests check that
claim by brute force on small matrices, show that the margin is tight (a
perturbation just past it can flip the matching), and check the near-tie
certificate."""
import numpy as np
import pytest

import oracle
from tests.parity import certify_near_tie, relative_margin


def _greedy(S):
    return oracle.greedy_match(np.asarray(S, np.float64))[0]


@pytest.mark.parametrize("seed", range(12))
def test_perturbations_inside_half_the_margin_keep_the_matching(seed):
    rng = np.random.default_rng(seed)
    nB, nA = rng.integers(2, 9, size=2)
    S = rng.random((nB, nA)) ** 3
    m0 = _greedy(S)
    m = relative_margin(S, m0, 0.0)
    assert 0.0 < m <= 1.0
    eps = 0.49 * m
    for _ in range(200):
        E = rng.uniform(-eps, eps, size=S.shape)
        assert np.array_equal(_greedy(S * (1.0 + E)), m0)


def test_margin_is_tight():
    # row 0: pick (0,0) = 1.0, rival (0,1) = 0.9 (column 1 free at that pick)
    S = np.array([[1.0, 0.9], [0.5, 0.1]])
    m0 = _greedy(S)
    assert m0.tolist() == [0, 1]
    m = relative_margin(S, m0, 0.0)
    assert abs(m - 0.1) < 1e-15
    # moving both entries by a relative 0.06 (> m/2) in opposite directions swaps them
    T = S.copy()
    T[0, 0] *= 1 - 0.06
    T[0, 1] *= 1 + 0.06
    assert _greedy(T).tolist() != m0.tolist()


def test_rivals_only_count_while_their_line_is_free():
    # (1,1) = 0.95 trails the first pick (0,0) = 1.0 but shares neither its row
    # nor its column; (1,0) = 0.2 shares column 0 but row 1 is matched later
    # by (1,1) (rank 2 after (0,0)), so it is a rival of (0,0): margin 0.8
    S = np.array([[1.0, 0.1], [0.2, 0.95]])
    m0 = _greedy(S)
    assert m0.tolist() == [0, 1]
    # rivals of (0,0): (0,1) = 0.1 (column 1 matched later), (1,0) = 0.2 ->
    # 1 - 0.2; rivals of (1,1): none left (row 0 and column 0 already taken)
    assert abs(relative_margin(S, m0, 0.0) - 0.8) < 1e-15


def test_exact_ties_and_tiny_picks_have_zero_margin():
    S = np.full((3, 3), 1 / 3)
    assert relative_margin(S, _greedy(S), 0.0) == 0.0
    S = np.array([[1.0, 0.0], [0.0, 1e-40]])
    # the second pick has no rival left: the margin comes from the first
    assert relative_margin(S, _greedy(S), 1e-38) == 1.0
    S = np.array([[1e-40, 5e-41], [0.0, 0.0]])
    assert relative_margin(S, _greedy(S), 1e-38) == 0.0


def test_no_rival_gives_infinity():
    assert np.isinf(relative_margin(np.array([[0.7]]), np.array([0]), 0.0))


@pytest.mark.parametrize("seed", range(6))
def test_certificate_accepts_near_tie_flips_and_rejects_wrong_picks(seed):
    rng = np.random.default_rng(100 + seed)
    S = rng.random((6, 6))
    S[2, 3] = S[2, 4] = 0.999          # an exact tie in row 2
    eps = 1e-6
    flipped = S * (1.0 + rng.uniform(-eps, eps, size=S.shape))
    mf = _greedy(flipped)
    certify_near_tie(flipped, mf, S, 2 * eps, 0.0)
    # a matching that is not greedy on S at all fails the certificate
    wrong = np.array([(int(_greedy(S)[i]) + 1) % 6 for i in range(6)])
    with pytest.raises(AssertionError):
        certify_near_tie(S, wrong, S, 2 * eps, 0.0)
