"""Plain FP64 CPU oracle of the damped IsoRank measure.

TEST INFRASTRUCTURE, like the rest of `oracle/`: only `tests/`,
`__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may import
it; it shares no code with the HIP library.

Table 1, row "Iso", writes the IsoRank measure in its full form as the
solution x of (I - alpha Q x P) x = rhs: the identity minus alpha times the
Kronecker product of the two transition matrices.  IsoRank, the method the
row cites, fixes the parts the table leaves out: the product-graph operator
has every column scaled to sum to one, the right-hand side is (1 - alpha) E
for a prior E over node pairs with unit sum, and 0 <= alpha < 1.

Readings where the paper is silent (each is listed in the design notes of
the repository):

* Operator.  The coupled operator of the undamped measure,
  M = B (x) A + B^T (x) A^T on the row-major vec of X (n_B x n_A), with its
  columns scaled to unit sum: M_hat = M D^-1, D = diag(column sums of M); a
  column that sums to zero stays zero.  Column (u, v) of M sums to
      d_uv = c^B_u c^A_v + r^B_u r^A_v
  (c = column sums, r = row sums of the transition matrices), so
  M_hat vec(X) = vec(B Z A^T + B^T Z A) with Z = X / d entry by entry (0
  where d = 0).  For symmetric 0/1 adjacency matrices M_hat is IsoRank's
  own matrix, 1 / (|N(u)| |N(v)|) between neighbouring node pairs.  M_hat is
  non-negative with column sums at most 1, so ||alpha M_hat||_1 <= alpha < 1
  and I - alpha M_hat is invertible.
* Prior.  E = the caller's non-negative prior (n_B x n_A) divided by its
  sum, or the uniform 1 / (n_A n_B).
* Solution.  The fixed-point iteration x_0 = E,
  x_k = alpha M_hat x_{k-1} + (1 - alpha) E, a contraction with factor alpha
  in the 1-norm; it stops at the first k with
  delta_k = ||x_k - x_{k-1}||_1 < tol, or at k = max_iter.  Then
  ||x_k - x*||_1 <= alpha delta_k / (1 - alpha).
* Output.  S = x_k / ||x_k||_F (n_B x n_A), so that S, the greedy matching
  and the score are read as for the undamped measure; nu = ||x_k||_F.

Floating point: float64; numpy products and sums are the library
primitives; nothing is blocked, fused or reordered.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .cfsim_ref import CONVERGED, HIT_MAX_ITER, PairResult, apply_operator, greedy_match


def _dense(X) -> np.ndarray:
    return X.toarray() if sp.issparse(X) else np.asarray(X, np.float64)


def column_sums(A, B) -> np.ndarray:
    """d (n_B x n_A): the column sums of M = B (x) A + B^T (x) A^T, entry
    (u, v) for column (u, v)."""
    A, B = _dense(A), _dense(B)
    cA, rA = A.sum(axis=0), A.sum(axis=1)
    cB, rB = B.sum(axis=0), B.sum(axis=1)
    return np.outer(cB, cA) + np.outer(rB, rA)


def apply_normalised(A, B, X: np.ndarray, d: np.ndarray | None = None) -> np.ndarray:
    """M_hat vec(X) as an n_B x n_A matrix: M applied to X / d (0 where d = 0)."""
    if d is None:
        d = column_sums(A, B)
    pos = d > 0
    Z = np.zeros_like(X, dtype=np.float64)
    Z[pos] = X[pos] / d[pos]
    return apply_operator(A, B, Z)


def prior_of(nA: int, nB: int, prior=None) -> np.ndarray:
    """E (n_B x n_A, unit sum): the uniform prior, or the caller's scaled."""
    if prior is None:
        return np.full((nB, nA), 1.0 / (nA * nB))
    E = np.asarray(prior, np.float64)
    if E.shape != (nB, nA):
        raise ValueError("prior must be n_B x n_A")
    total = E.sum()
    if not (np.isfinite(E).all() and (E >= 0).all() and total > 0):
        raise ValueError("prior must be finite, non-negative and not all zero")
    return E / total


def damped_iteration(A, B, alpha: float, prior=None, max_iter: int = 200, tol: float = 1e-12,
                     keep_iterates: bool = False):
    """The fixed-point iteration of (I - alpha M_hat) x = (1 - alpha) E.

    Returns (S, nu, delta, iters, status[, iterates]): S = x_k / ||x_k||_F,
    nu = ||x_k||_F, delta = ||x_k - x_{k-1}||_1, iters = k.
    """
    if not (0.0 <= alpha < 1.0):
        raise ValueError("alpha must lie in [0, 1)")
    nA, nB = A.shape[0], B.shape[0]
    E = prior_of(nA, nB, prior)
    d = column_sums(A, B)
    x = E.copy()
    iterates = [x]
    delta = np.inf
    status = HIT_MAX_ITER
    iters = 0
    for k in range(1, max_iter + 1):
        x_new = alpha * apply_normalised(A, B, x, d) + (1.0 - alpha) * E
        delta = float(np.abs(x_new - x).sum())
        x = x_new
        iters = k
        if keep_iterates:
            iterates.append(x)
        if delta < tol:
            status = CONVERGED
            break
    nu = float(np.linalg.norm(x))
    out = (x / nu, nu, delta, iters, status)
    return out + (iterates,) if keep_iterates else out


def score_pair_damped(A, B, alpha: float, prior=None, max_iter: int = 200, tol: float = 1e-12) -> PairResult:
    """Damped measure of one pair: S, nu, delta, iters, status, greedy
    matching and score (the sum of S over the matching)."""
    S, nu, delta, iters, status = damped_iteration(A, B, alpha, prior, max_iter, tol)
    match, score = greedy_match(S)
    return PairResult(S, nu, delta, iters, status, match, score)
