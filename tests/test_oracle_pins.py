"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test fixes the oracle to something independent of its own code: an
eigen-decomposition closed form, a singular-value special case (HITS),
a hand-derived fixed point, library routines (scipy zoom), brute force,
invariants the mathematics guarantees, and finite differences.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from cfgsynth import Grammar, make_cfg
from oracle import cfsim_ref as ref


def _rand_digraph(rng, n, density=0.4, self_loops=True):
    X = rng.random((n, n)) * (rng.random((n, n)) < density)
    if not self_loops:
        np.fill_diagonal(X, 0.0)
    if not (X > 0).any():
        X[0, n - 1] = 1.0
    return X


def _kron_operator(A, B):
    """The Kronecker operator acting on row-major vec(S), S = n_B x n_A."""
    return np.kron(B, A) + np.kron(B.T, A.T)


def _closed_form_iterate(A, B, K):
    """vec(S_K) proportional to sum_i (lambda_i/rho)^K (v_i^T s0) v_i."""
    M = _kron_operator(A, B)
    lam, V = np.linalg.eigh(M)          # M is symmetric
    rho = np.abs(lam).max()
    s0 = np.full(M.shape[0], 1.0 / np.sqrt(M.shape[0]))
    x = V @ (((lam / rho) ** K) * (V.T @ s0))
    x /= np.linalg.norm(x)
    return x.reshape(B.shape[0], A.shape[0])


def _cfg_matrix(n, seed, counts="trip"):
    g = make_cfg(n, Grammar(counts=counts), seed=seed)
    return oracle.transition_matrix(g.n, g.src, g.dst, g.count), g


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("K", [1, 2, 3, 7, 30, 200])
def test_fixed_K_iterate_equals_eigen_closed_form(seed, K):
    rng = np.random.default_rng(seed)
    A = _rand_digraph(rng, int(rng.integers(2, 7)))
    B = _rand_digraph(rng, int(rng.integers(2, 6)))
    S, nu, delta, iters, status = oracle.coupled_iteration(A, B, max_iter=K, tol=-1.0)
    assert iters == K and status == oracle.HIT_MAX_ITER
    np.testing.assert_allclose(S, _closed_form_iterate(A, B, K), atol=1e-10, rtol=0)


@pytest.mark.parametrize("seed", range(4))
def test_cfg_pairs_equal_eigen_closed_form(seed):
    A, _ = _cfg_matrix(9, 100 + seed)
    B, _ = _cfg_matrix(7, 200 + seed)
    for K in (2, 5, 40, 200):
        S = oracle.coupled_iteration(A, B, max_iter=K, tol=-1.0)[0]
        np.testing.assert_allclose(S, _closed_form_iterate(A, B, K), atol=1e-10, rtol=0)


def test_limit_is_perron_vector_of_positive_operator():
    rng = np.random.default_rng(7)
    A = rng.random((5, 5)) + 0.1
    B = rng.random((4, 4)) + 0.1
    S, nu, delta, iters, status = oracle.coupled_iteration(A, B, max_iter=500, tol=1e-14)
    assert status == oracle.CONVERGED
    lam, V = np.linalg.eigh(_kron_operator(A, B))
    v = V[:, np.argmax(lam)]
    v = v * np.sign(v.sum())
    np.testing.assert_allclose(S.ravel(), v, atol=1e-12)
    assert abs(nu - lam.max()) < 1e-12 * lam.max()


def test_nu_tends_to_spectral_radius_on_cfg():
    A, _ = _cfg_matrix(10, 5, counts="uniform")
    B, _ = _cfg_matrix(8, 6, counts="uniform")
    S, nu, *_ = oracle.coupled_iteration(A, B, max_iter=4000, tol=1e-13)
    rho = np.abs(np.linalg.eigvalsh(_kron_operator(A, B))).max()
    assert abs(nu - rho) < 1e-6 * rho


# ---------------------------------------------------------------- P2 (HITS)
@pytest.mark.parametrize("seed", range(4))
def test_two_node_path_gives_hits_vectors(seed):
    rng = np.random.default_rng(seed)
    A = rng.random((6, 6)) * (rng.random((6, 6)) < 0.7) + 0.05 * np.eye(6)
    B = np.array([[0.0, 1.0], [0.0, 0.0]])
    S, nu, delta, iters, status = oracle.coupled_iteration(A, B, max_iter=4000, tol=1e-15)
    U, sig, Vt = np.linalg.svd(A)
    assert sig[0] > 1.05 * sig[1]
    u1, v1 = U[:, 0], Vt[0]
    alpha, beta = u1.sum(), v1.sum()
    expect = np.vstack([alpha * u1, beta * v1]) / np.hypot(alpha, beta)
    np.testing.assert_allclose(S, expect, atol=1e-11)
    assert abs(nu - sig[0]) < 1e-11


# ---------------------------------------------------------------- P3
def test_self_loop_singleton_is_symmetrised_power_iteration():
    A, _ = _cfg_matrix(11, 3)
    B = np.array([[1.0]])
    for K in (3, 10, 60):
        S = oracle.coupled_iteration(A, B, max_iter=K, tol=-1.0)[0]
        H = A + A.T
        lam, V = np.linalg.eigh(H)
        rho = np.abs(lam).max()
        x = V @ (((lam / rho) ** K) * (V.T @ np.ones(11)))
        x /= np.linalg.norm(x)
        np.testing.assert_allclose(S.ravel(), x, atol=1e-11)


# ---------------------------------------------------------------- hand example
def test_hand_worked_two_node_path_pair():
    # Y = diag(S11, S00) for A = B = one jump 0 -> 1, so from the uniform start
    # S_1 = I/sqrt(2) = S_2 = ... ; the first even test (k=2) compares with S_0
    # and fails, the second (k=4) sees no change.
    P = np.array([[0.0, 1.0], [0.0, 0.0]])
    r = oracle.score_pair(P, P, max_iter=200, tol=1e-12)
    np.testing.assert_allclose(r.S, np.eye(2) / np.sqrt(2.0), atol=2e-16, rtol=0)
    assert r.iters == 4 and r.status == oracle.CONVERGED
    assert r.match.tolist() == [0, 1]
    assert r.score == pytest.approx(np.sqrt(2.0), abs=1e-15)
    # from S_1 on, Y = diag(1, 1)/sqrt(2) has norm 1
    assert r.nu == pytest.approx(1.0, abs=1e-15)


def test_self_loop_singletons_score_one():
    r = oracle.score_pair(np.array([[1.0]]), np.array([[1.0]]))
    assert r.S.tolist() == [[1.0]] and r.score == 1.0 and r.iters == 2
    assert r.status == oracle.CONVERGED


# ---------------------------------------------------------------- P4 invariants
@pytest.fixture(scope="module")
def cfg_pair():
    A, ga = _cfg_matrix(13, 11)
    B, gb = _cfg_matrix(9, 12)
    return A, B


def test_unit_norm_nonnegative(cfg_pair):
    A, B = cfg_pair
    r = oracle.score_pair(A, B)
    assert abs(np.linalg.norm(r.S) - 1.0) < 1e-14
    assert (r.S >= 0).all()
    assert 0 < r.score <= np.sqrt(min(A.shape[0], B.shape[0])) + 1e-12


def test_self_pair_is_symmetric(cfg_pair):
    A, _ = cfg_pair
    S = oracle.score_pair(A, A).S
    np.testing.assert_allclose(S, S.T, atol=1e-14)


def test_swap_transposes(cfg_pair):
    A, B = cfg_pair
    r1 = oracle.score_pair(A, B)
    r2 = oracle.score_pair(B, A)
    np.testing.assert_allclose(r2.S, r1.S.T, atol=1e-13)
    assert r1.iters == r2.iters
    assert abs(r1.score - r2.score) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_permutation_equivariance(cfg_pair, seed):
    A, B = cfg_pair
    rng = np.random.default_rng(seed)
    pa, pb = rng.permutation(A.shape[0]), rng.permutation(B.shape[0])
    PA, PB = np.eye(A.shape[0])[pa], np.eye(B.shape[0])[pb]
    S = oracle.coupled_iteration(A, B, 60, -1.0)[0]
    Sp = oracle.coupled_iteration(PA @ A @ PA.T, PB @ B @ PB.T, 60, -1.0)[0]
    np.testing.assert_allclose(Sp, PB @ S @ PA.T, atol=1e-13)


def test_power_of_two_scaling_is_bit_exact(cfg_pair):
    A, B = cfg_pair
    S = oracle.coupled_iteration(A, B, 50, -1.0)[0]
    S2 = oracle.coupled_iteration(4.0 * A, 0.5 * B, 50, -1.0)[0]
    np.testing.assert_array_equal(S, S2)
    S3 = oracle.coupled_iteration(3.7 * A, B, 50, -1.0)[0]
    np.testing.assert_allclose(S, S3, atol=1e-14)


def test_even_step_test_handles_oscillation():
    # A = path 0 -> 1 -> 2, B = one self-loop node: M = A + A^T has eigenvalues
    # +-sqrt(2) and 0, and the iterates alternate exactly between
    # (1, 2, 1)/sqrt(6) (odd k) and the uniform start (even k).  Only the
    # even-step test (S_2 against S_0) sees convergence.
    P = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0]])
    one = np.array([[1.0]])
    S1 = oracle.coupled_iteration(P, one, 1, -1.0)[0]
    np.testing.assert_allclose(S1, [[1 / np.sqrt(6), 2 / np.sqrt(6), 1 / np.sqrt(6)]], atol=1e-15)
    r = oracle.score_pair(P, one, max_iter=200, tol=1e-12)
    assert r.iters == 2 and r.status == oracle.CONVERGED
    np.testing.assert_allclose(r.S, np.full((1, 3), 1 / np.sqrt(3)), atol=1e-15)
    assert r.delta < 1e-15
    assert r.match.tolist() == [0]      # three-way tie -> lowest index
    r3 = oracle.coupled_iteration(P, one, 3, -1.0)
    assert r3[3] == 3 and np.linalg.norm(r3[0] - S1) < 1e-15


def test_degenerate_edgeless_graph():
    A, _ = _cfg_matrix(5, 2)
    Z = np.zeros((4, 4))
    r = oracle.score_pair(A, Z)
    assert r.status == oracle.DEGENERATE and r.iters == 0 and r.nu == 0.0
    np.testing.assert_array_equal(r.S, np.full((4, 5), 1 / np.sqrt(20)))
    assert r.match.tolist() == [0, 1, 2, 3]


# ---------------------------------------------------------------- transition matrices
def test_transition_matrix_is_right_stochastic():
    g = make_cfg(40, Grammar(counts="trip"), seed=3)
    P = oracle.transition_matrix(g.n, g.src, g.dst, g.count)
    rows = P.sum(axis=1)
    assert abs(rows[-1]) == 0.0                       # STOP row
    assert np.all(np.abs(rows[:-1] - 1.0) < 1e-15)
    Ps = oracle.transition_matrix_sparse(g.n, g.src, g.dst, g.count).toarray()
    np.testing.assert_allclose(Ps, P, atol=1e-16)


def test_transition_matrix_hand_example():
    # node 0 jumps to 1 (30 times) and 2 (10 times); 1 -> 2 (5); 2 is STOP
    P = oracle.transition_matrix(3, [0, 0, 1], [1, 2, 2], [30, 10, 5])
    np.testing.assert_array_equal(P, [[0, 0.75, 0.25], [0, 0, 1], [0, 0, 0]])


# ---------------------------------------------------------------- P5 resize
@pytest.mark.parametrize("m,M", [(3, 7), (5, 16), (12, 16), (1, 4), (2, 3), (8, 128), (40, 41)])
def test_resize_matches_scipy_zoom_order1(m, M):
    X = np.random.default_rng(m * 1000 + M).random((m, m))
    Z = ndi.zoom(X, M / m, order=1, grid_mode=False, mode="nearest")
    assert Z.shape == (M, M)
    np.testing.assert_allclose(oracle.resize_bilinear(X, M), Z, atol=1e-15)


def test_resize_keeps_corners_and_identity():
    X = np.random.default_rng(1).random((6, 6))
    R = oracle.resize_bilinear(X, 11)
    for (p, q), (r, c) in {(0, 0): (0, 0), (0, 10): (0, 5), (10, 0): (5, 0), (10, 10): (5, 5),
                           (2, 4): (1, 2)}.items():
        assert R[p, q] == pytest.approx(X[r, c], abs=1e-15)
    np.testing.assert_array_equal(oracle.resize_bilinear(X, 6), X)


def test_resize_sparse_equals_dense():
    A, g = _cfg_matrix(30, 9)
    Ad = oracle.resize_bilinear(A, 47)
    As = oracle.resize_bilinear(oracle.transition_matrix_sparse(g.n, g.src, g.dst, g.count), 47)
    np.testing.assert_allclose(As.toarray(), Ad, atol=1e-15)


# ---------------------------------------------------------------- P6 matching
def _naive_greedy(S):
    S = S.copy()
    nB, nA = S.shape
    avail = np.ones_like(S, bool)
    match = [-1] * nB
    for _ in range(min(nA, nB)):
        best, bi, bj = -np.inf, -1, -1
        for i in range(nB):
            for j in range(nA):
                if avail[i, j] and S[i, j] > best:
                    best, bi, bj = S[i, j], i, j
        match[bi] = bj
        avail[bi, :] = False
        avail[:, bj] = False
    return match


def _locally_dominant(S):
    """Parallel rounds: match every (i, j) where j is row i's best free column
    and i is column j's best free row (order: value desc, flat index asc)."""
    nB, nA = S.shape
    rfree, cfree = np.ones(nB, bool), np.ones(nA, bool)
    match = [-1] * nB
    key = lambda i, j: (-S[i, j], i * nA + j)
    while rfree.any() and cfree.any():
        rbest = {i: min((j for j in range(nA) if cfree[j]), key=lambda j: key(i, j))
                 for i in range(nB) if rfree[i]}
        cbest = {j: min((i for i in range(nB) if rfree[i]), key=lambda i: key(i, j))
                 for j in range(nA) if cfree[j]}
        for i, j in rbest.items():
            if cbest[j] == i:
                match[i] = j
        for i, j in rbest.items():
            if cbest[j] == i:
                rfree[i] = False
                cfree[j] = False
    return match


@pytest.mark.parametrize("seed", range(12))
def test_greedy_equals_naive_and_locally_dominant(seed):
    rng = np.random.default_rng(seed)
    nB, nA = int(rng.integers(1, 9)), int(rng.integers(1, 9))
    # integer values force many exact ties
    S = rng.integers(0, 4, size=(nB, nA)).astype(float)
    match, score = oracle.greedy_match(S)
    assert match.tolist() == _naive_greedy(S)
    assert match.tolist() == _locally_dominant(S)
    assert score == sum(S[i, j] for i, j in enumerate(match) if j >= 0)


@pytest.mark.parametrize("seed", range(6))
def test_greedy_pick_property_brute_force(seed):
    """Every pick is the maximum (value desc, index asc) of all entries disjoint
    from the earlier picks, and the matching saturates the smaller side."""
    rng = np.random.default_rng(100 + seed)
    nB, nA = int(rng.integers(1, 7)), int(rng.integers(1, 7))
    S = np.round(rng.random((nB, nA)), 1)
    match, _ = oracle.greedy_match(S)
    picks = sorted(((i, j) for i, j in enumerate(match) if j >= 0),
                   key=lambda e: (-S[e], e[0] * nA + e[1]))
    assert len(picks) == min(nA, nB)
    used_r, used_c = set(), set()
    for (i, j) in picks:
        cands = [(a, b) for a in range(nB) for b in range(nA) if a not in used_r and b not in used_c]
        best = min(cands, key=lambda e: (-S[e], e[0] * nA + e[1]))
        assert best == (i, j)
        used_r.add(i)
        used_c.add(j)


# ---------------------------------------------------------------- P7 gradients
def _frozen_score(A, B, K, match):
    S = oracle.coupled_iteration(A, B, max_iter=K, tol=-1.0)[0]
    return sum(S[i, j] for i, j in enumerate(match) if j >= 0)


@pytest.mark.parametrize("seed", range(3))
def test_backward_matches_central_differences(seed):
    A, ga = _cfg_matrix(7, 300 + seed)
    B, gb = _cfg_matrix(6, 400 + seed)
    K = 30
    r = oracle.score_pair(A, B, max_iter=K, tol=-1.0)
    dA, dB = oracle.backward(A, B, K, r.match)
    h = 1e-6
    for X, dX, g, which in ((A, dA, ga, "A"), (B, dB, gb, "B")):
        for e in range(g.nnz):
            p, q = int(g.src[e]), int(g.dst[e])
            Xp, Xm = X.copy(), X.copy()
            Xp[p, q] += h
            Xm[p, q] -= h
            if which == "A":
                fd = (_frozen_score(Xp, B, K, r.match) - _frozen_score(Xm, B, K, r.match)) / (2 * h)
            else:
                fd = (_frozen_score(A, Xp, K, r.match) - _frozen_score(A, Xm, K, r.match)) / (2 * h)
            assert abs(fd - dX[p, q]) < 1e-8 * max(1.0, abs(fd)), (which, e, fd, dX[p, q])


def test_backward_tends_to_implicit_function_gradient():
    rng = np.random.default_rng(5)
    A = rng.random((4, 4)) + 0.2
    B = rng.random((3, 3)) + 0.2
    K = 400
    r = oracle.score_pair(A, B, max_iter=K, tol=-1.0)
    dA, dB = oracle.backward(A, B, K, r.match)
    M = _kron_operator(A, B)
    lam, V = np.linalg.eigh(M)
    rho = lam.max()
    s = r.S.ravel()
    g = np.zeros_like(s)
    for i, j in enumerate(r.match):
        if j >= 0:
            g[i * A.shape[0] + j] = 1.0
    keep = lam < rho - 1e-9
    P = (V[:, keep] / (rho - lam[keep])) @ V[:, keep].T
    w = P @ (g - s * (s @ g))
    W = w.reshape(r.S.shape)
    S = r.S
    np.testing.assert_allclose(dA, W.T @ B @ S + S.T @ B @ W, atol=1e-10)
    np.testing.assert_allclose(dB, W @ A @ S.T + S @ A @ W.T, atol=1e-10)


def test_edge_gradients_gather():
    dX = np.arange(9.0).reshape(3, 3)
    assert oracle.edge_gradients(dX, [0, 2, 1], [1, 0, 1]).tolist() == [1.0, 6.0, 4.0]


# ---------------------------------------------------------------- top-k
def test_topk_ties_go_to_lower_index():
    s = np.array([0.5, 0.9, 0.9, np.nan, 0.1, 0.9])
    idx, val = oracle.topk(s, 4)
    assert idx.tolist() == [1, 2, 5, 0]
    assert val.tolist() == [0.9, 0.9, 0.9, 0.5]
    assert oracle.topk(s, 6)[0].tolist() == [1, 2, 5, 0, 4, 3]


# ---------------------------------------------------------------- sparse == dense
def test_sparse_oracle_equals_dense():
    A, ga = _cfg_matrix(40, 21)
    B, gb = _cfg_matrix(33, 22)
    As = oracle.transition_matrix_sparse(ga.n, ga.src, ga.dst, ga.count)
    Bs = oracle.transition_matrix_sparse(gb.n, gb.src, gb.dst, gb.count)
    r1 = oracle.score_pair(A, B, 80, -1.0)
    r2 = oracle.score_pair(As, Bs, 80, -1.0)
    np.testing.assert_allclose(r2.S, r1.S, atol=1e-14)
    assert r1.match.tolist() == r2.match.tolist()
