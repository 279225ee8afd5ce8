"""Plain FP64 CPU oracle of the five elementwise distances of Table 1.

TEST INFRASTRUCTURE, like the rest of `oracle/`: only `tests/`,
`__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may import
it; it shares no code with the HIP library.

Section 4 (Methodology) and Section 4.1 (Bilinear Interpolation) bring the
two transition matrices of a pair to a common size M = max(n_A, n_B): the
smaller one is upsampled by an order-1 spline, the larger one is kept.
Section 4.2 (Pairwise Comparison) then compares the pair by one measure of
Table 1.  Apart from "Iso" (the coupled iteration in `cfsim_ref`), the
measures are elementwise over the two scaled matrices, read as vectors
x = vec(P_A') and y = vec(P_B') of n = M^2 entries:

    Euclidean   sqrt( sum |x_i - y_i|^2 )
    Manhattan   sum |x_i - y_i|
    Minkowski   ( sum |x_i - y_i|^p )^(1/p)
    Jaccard     sum (x_i - y_i)^2 / ( sum x_i^2 + sum y_i^2 - sum x_i y_i )
    Cosine      1 - sum x_i y_i / ( sqrt(sum x_i^2) sqrt(sum y_i^2) )

Readings where the paper is silent:
* The vectors are the scaled transition matrices themselves (the objects
  Section 4.2 says are compared), flattened in one common order; all five
  measures are symmetric in (x, y) and invariant under a common reordering,
  so neither the order nor which graph is called A matters.
* Minkowski order: not given; p = 3 by default (p = 1 and p = 2 would repeat
  Manhattan and Euclidean).  Any finite p >= 1 is accepted.
* Jaccard with x = y = 0: the denominator is 0 only then (it is at least
  (sum x^2 + sum y^2) / 2); the distance is 0, the distance of a graph to
  itself.  Cosine with a zero vector is undefined: NaN.

Floating point: float64, numpy sums over the flattened arrays; nothing is
blocked or reordered beyond what numpy's sum does.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .cfsim_ref import common_size

NAMES = ("euclidean", "manhattan", "minkowski", "jaccard", "cosine")
DEFAULT_P = 3.0


def scaled_pair(A, B):
    """The two transition matrices at the common size M (Section 4, 4.1),
    dense float64 M x M arrays."""
    A2, B2 = common_size(A, B, "bilinear")
    dense = (lambda X: X.toarray() if sp.issparse(X) else np.asarray(X, np.float64))
    return dense(A2), dense(B2)


def elementwise_distances(x, y, p: float = DEFAULT_P) -> np.ndarray:
    """Table 1's five elementwise measures of two equal-length vectors, in the
    order of NAMES."""
    x = np.asarray(x, np.float64).ravel()
    y = np.asarray(y, np.float64).ravel()
    if x.shape != y.shape:
        raise ValueError("x and y must have the same number of entries")
    if not (p >= 1.0 and np.isfinite(p)):
        raise ValueError("the Minkowski order p must be finite and >= 1")
    d = np.abs(x - y)
    sxx = np.sum(x * x)
    syy = np.sum(y * y)
    sxy = np.sum(x * y)
    euclidean = np.sqrt(np.sum(d ** 2))
    manhattan = np.sum(d)
    minkowski = np.sum(d ** p) ** (1.0 / p)
    denom = sxx + syy - sxy
    jaccard = np.sum(d ** 2) / denom if denom > 0 else 0.0
    cosine = 1.0 - sxy / (np.sqrt(sxx) * np.sqrt(syy)) if sxx > 0 and syy > 0 else np.nan
    return np.array([euclidean, manhattan, minkowski, jaccard, cosine], np.float64)


def pair_distances(A, B, p: float = DEFAULT_P) -> np.ndarray:
    """The five measures of one pair of transition matrices (n_A x n_A and
    n_B x n_B): scale to the common size, flatten, compare."""
    A2, B2 = scaled_pair(A, B)
    return elementwise_distances(A2, B2, p)
