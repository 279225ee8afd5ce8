"""Plain FP64 CPU oracle of the CFG-pair similarity.

TEST INFRASTRUCTURE.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import, call or execute this module.
It shares no code with the HIP library and imports nothing from it.

Method (Lim, Norris & Malony, "A Similarity Measure for GPU Kernel Subgraph
Matching", arXiv 1707.02423):

* Section 3 (Background), "Transition probability": each CFG becomes a right-stochastic
  transition matrix, P[i, j] = Pr(j | i), every non-empty row sums to 1.
* Section 4 (Methodology) and Section 4.1 (Bilinear Interpolation): the smaller matrix is interpolated up to the
  larger size with an order-1 (bilinear) spline before comparison.
* Table 1, row "Iso", and Section 4.2 (Pairwise Comparison): graphs are compared by the IsoRank
  solution of the Kronecker operator of the two matrices.

Readings taken where the paper is silent or garbled (each is listed in the
design notes of the repository):

* Operator: for directed graphs the coupled operator is
  M = B (x) A + B^T (x) A^T acting on the row-major vec of S (n_B x n_A),
  i.e. Y = B S A^T + B^T S A; alpha = 1, no prior vector.  The IsoRank
  fixed point is reached by normalised power iteration.
* Start S_0 = 1/sqrt(n_A n_B) everywhere; Frobenius normalisation each step.
* Stopping: only at even k, delta_k = ||S_k - S_{k-2}||_F < tol, else at
  k = max_iter; the iterate at that k is returned.  (M has the eigenvalue
  -rho whenever the product graph is bipartite, so odd and even iterates
  can oscillate.)
* Degenerate input: if A or B has no positive weight, M = 0; S_0 is
  returned with iters = 0 and the DEGENERATE status.
* Score: greedy node matching on S in the total order (value descending,
  row-major flat index ascending); score = sum of matched entries of S.
* Resize: corner-aligned order-1 spline, X'[p, q] sampled at
  (p (m-1)/(M-1), q (m-1)/(M-1)); no renormalisation afterwards.

Floating point: everything is float64; numpy / scipy matrix products and
norms serve as library primitives; nothing is blocked, fused or reordered.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

CONVERGED = 1
HIT_MAX_ITER = 2
DEGENERATE = 4
INVALID_INPUT = 8


# --------------------------------------------------------------------------
# Step a1: transition-probability matrices (Section 3, "Transition probability")
# --------------------------------------------------------------------------
def transition_matrix(n: int, src, dst, count) -> np.ndarray:
    """Dense right-stochastic matrix of one CFG.

    P[i, j] = c_ij / sum_j' c_ij'.  Repeated (i, j) jumps add up.  A row
    whose counts sum to zero (the STOP node) stays all zero.
    """
    C = np.zeros((n, n), dtype=np.float64)
    np.add.at(C, (np.asarray(src, np.int64), np.asarray(dst, np.int64)),
              np.asarray(count, np.float64))
    row = C.sum(axis=1)
    P = np.zeros_like(C)
    nz = row > 0
    P[nz] = C[nz] / row[nz, None]
    return P


def transition_matrix_sparse(n: int, src, dst, count) -> sp.csr_matrix:
    """Same as `transition_matrix`, as a scipy CSR matrix (large graphs)."""
    C = sp.csr_matrix((np.asarray(count, np.float64),
                       (np.asarray(src, np.int64), np.asarray(dst, np.int64))),
                      shape=(n, n))
    C.sum_duplicates()
    row = np.asarray(C.sum(axis=1)).ravel()
    inv = np.zeros(n)
    inv[row > 0] = 1.0 / row[row > 0]
    return sp.csr_matrix(sp.diags(inv) @ C)


# --------------------------------------------------------------------------
# Step a2: scale to a common size (Section 4, Section 4.1)
# --------------------------------------------------------------------------
def _interp_matrix(m: int, M: int):
    """M x m matrix of 1-D linear interpolation at p (m-1)/(M-1)."""
    rows, cols, vals = [], [], []
    for p in range(M):
        num = p * (m - 1)
        r0 = num // (M - 1) if M > 1 else 0
        f = (num - r0 * (M - 1)) / (M - 1) if M > 1 else 0.0
        r1 = min(r0 + 1, m - 1)
        rows += [p, p]
        cols += [r0, r1]
        vals += [1.0 - f, f]
    return sp.csr_matrix((vals, (rows, cols)), shape=(M, m))


def resize_bilinear(X, M: int):
    """Bilinear (order-1 spline) upsampling of an m x m matrix to M x M.

    Linear interpolation along rows, then along columns: X' = R X R^T.
    The result is dense for dense X and sparse for sparse X.
    """
    m = X.shape[0]
    if m == M:
        return X.copy()
    if m > M:
        raise ValueError("resize only enlarges the smaller matrix")
    R = _interp_matrix(m, M)
    if sp.issparse(X):
        return sp.csr_matrix(R @ X @ R.T)
    Rd = R.toarray()
    return Rd @ X @ Rd.T


# --------------------------------------------------------------------------
# Steps a3-a6: coupled iteration (Table 1 "Iso", Section 4.2)
# --------------------------------------------------------------------------
def apply_operator(A, B, S: np.ndarray) -> np.ndarray:
    """Y = B S A^T + B^T S A, the Kronecker operator (B (x) A + B^T (x) A^T)
    on the row-major vec of S (S is n_B x n_A)."""
    if sp.issparse(A) or sp.issparse(B):
        A = sp.csr_matrix(A)
        B = sp.csr_matrix(B)
        BS = np.asarray(B @ S)
        BtS = np.asarray(B.T @ S)
        return np.asarray(A @ BS.T).T + np.asarray(A.T @ BtS.T).T
    return B @ S @ A.T + B.T @ S @ A


def _has_positive(X) -> bool:
    if sp.issparse(X):
        return bool((X.data > 0).any())
    return bool((np.asarray(X) > 0).any())


def coupled_iteration(A, B, max_iter: int = 200, tol: float = 1e-12, keep_iterates: bool = False):
    """Normalised power iteration of the coupled operator.

    Returns (S, nu, delta, iters, status[, iterates, nus]) where nu is the
    norm of the last un-normalised update, delta the last even-step change
    (inf if none was taken), iters the number of updates applied.
    """
    nA, nB = A.shape[0], B.shape[0]
    S = np.full((nB, nA), 1.0 / np.sqrt(nA * nB))
    iterates, nus = [S], []
    if not (_has_positive(A) and _has_positive(B)):
        out = (S, 0.0, np.inf, 0, DEGENERATE)
        return out + (iterates, nus) if keep_iterates else out
    prev_even = S
    delta = np.inf
    status = HIT_MAX_ITER
    iters = 0
    nu = 0.0
    for k in range(1, max_iter + 1):
        Y = apply_operator(A, B, S)
        nu = float(np.linalg.norm(Y))
        S = Y / nu
        iters = k
        if keep_iterates:
            iterates.append(S)
            nus.append(nu)
        if k % 2 == 0:
            delta = float(np.linalg.norm(S - prev_even))
            prev_even = S
            if delta < tol:
                status = CONVERGED
                break
    out = (S, nu, delta, iters, status)
    return out + (iterates, nus) if keep_iterates else out


# --------------------------------------------------------------------------
# Step a7: score and node matching (Section 4.2; IsoRank's greedy extraction)
# --------------------------------------------------------------------------
def greedy_match(S: np.ndarray):
    """Greedy matching: repeatedly take the largest S[i, j] whose row and
    column are both unused; ties go to the smaller row-major flat index.

    Returns (match, score): match[i] = j or -1 for the n_B rows, and the sum
    of the matched entries taken in ascending row order.
    """
    nB, nA = S.shape
    flat = np.asarray(S, np.float64).ravel()
    order = np.lexsort((np.arange(flat.size), -flat))
    row_used = np.zeros(nB, bool)
    col_used = np.zeros(nA, bool)
    match = np.full(nB, -1, np.int32)
    need = min(nA, nB)
    got = 0
    for idx in order:
        i, j = divmod(int(idx), nA)
        if row_used[i] or col_used[j]:
            continue
        match[i] = j
        row_used[i] = True
        col_used[j] = True
        got += 1
        if got == need:
            break
    score = 0.0
    for i in range(nB):
        if match[i] >= 0:
            score += float(S[i, match[i]])
    return match, score


@dataclasses.dataclass
class PairResult:
    S: np.ndarray
    nu: float
    delta: float
    iters: int
    status: int
    match: np.ndarray
    score: float


def common_size(A, B, resize: str = "none"):
    """Apply the paper's scale-to-common-size step if requested."""
    if resize == "none" or A.shape[0] == B.shape[0]:
        return A, B
    if resize != "bilinear":
        raise ValueError(resize)
    M = max(A.shape[0], B.shape[0])
    if A.shape[0] < M:
        A = resize_bilinear(A, M)
    else:
        B = resize_bilinear(B, M)
    return A, B


def score_pair(A, B, max_iter: int = 200, tol: float = 1e-12, resize: str = "none") -> PairResult:
    """Steps a2-a7 for one pair (A: n_A x n_A, B: n_B x n_B)."""
    A, B = common_size(A, B, resize)
    S, nu, delta, iters, status = coupled_iteration(A, B, max_iter, tol)
    match, score = greedy_match(S)
    return PairResult(S, nu, delta, iters, status, match, score)


# --------------------------------------------------------------------------
# Step a10: reverse mode through the fixed number of updates
# --------------------------------------------------------------------------
def backward(A, B, iters: int, match: np.ndarray):
    """d(score)/dA and d(score)/dB (dense), with the update count and the
    matching held fixed (the almost-everywhere derivative).

    Forward: S_{k+1} = Y_k / nu_k, Y_k = B S_k A^T + B^T S_k A.
    Reverse, from G = indicator of the matching:
      Ybar = (G - S_{k+1} <S_{k+1}, G>) / nu_k
      dA  += Ybar^T B S_k + S_k^T B Ybar
      dB  += Ybar A S_k^T + S_k A Ybar^T
      G    = B^T Ybar A + B Ybar A^T
    """
    A = np.asarray(A.toarray() if sp.issparse(A) else A, np.float64)
    B = np.asarray(B.toarray() if sp.issparse(B) else B, np.float64)
    nA, nB = A.shape[0], B.shape[0]
    S, nu, delta, k_done, status, iterates, nus = coupled_iteration(
        A, B, max_iter=iters, tol=-1.0, keep_iterates=True)
    dA = np.zeros_like(A)
    dB = np.zeros_like(B)
    if status & DEGENERATE:
        return dA, dB
    G = np.zeros((nB, nA))
    for i in range(nB):
        if match[i] >= 0:
            G[i, match[i]] = 1.0
    for k in range(k_done - 1, -1, -1):
        Sk, Sk1 = iterates[k], iterates[k + 1]
        Ybar = (G - Sk1 * float(np.sum(Sk1 * G))) / nus[k]
        dA += Ybar.T @ B @ Sk + Sk.T @ B @ Ybar
        dB += Ybar @ A @ Sk.T + Sk @ A @ Ybar.T
        G = B.T @ Ybar @ A + B @ Ybar @ A.T
    return dA, dB


def edge_gradients(dX: np.ndarray, src, dst) -> np.ndarray:
    """Gradient with respect to each listed edge weight X[src[e], dst[e]]."""
    return dX[np.asarray(src, np.int64), np.asarray(dst, np.int64)].astype(np.float64)


# --------------------------------------------------------------------------
# Step a11: top-k of a score vector
# --------------------------------------------------------------------------
def topk(scores, k: int):
    """Indices and values of the k largest scores; ties go to the lower index;
    NaN counts as -inf."""
    s = np.asarray(scores, np.float64).copy()
    s[np.isnan(s)] = -np.inf
    order = np.lexsort((np.arange(s.size), -s))[:k]
    return order.astype(np.int32), s[order]
