"""Plain FP64 CPU oracle of Ward's hierarchical clustering.

TEST INFRASTRUCTURE, like the rest of `oracle/`: only `tests/`,
`__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may import
it; it shares no code with the HIP library.

Section 6.2 ("Clustering of Kernels") groups kernels by Ward's minimum
variance method: starting from one cluster per kernel, it repeatedly merges
the pair of clusters whose union increases the total within-cluster variance
least, the initial distance between two kernels being the squared Euclidean
distance of their feature vectors, d_ij = ||X_i - X_j||^2 (the features are
instruction mixes, graph structure and distance measures; here, whatever the
caller puts in X, e.g. each graph's row of the all-pairs score matrix).

Readings:
* Distances between clusters follow the Lance-Williams recurrence of Ward's
  method on squared Euclidean distances: merging i and j into u,
      d(k, u) = ((n_i + n_k) d(k, i) + (n_j + n_k) d(k, j) - n_k d(i, j))
                / (n_i + n_j + n_k),
  which keeps d(a, b) = 2 n_a n_b / (n_a + n_b) ||c_a - c_b||^2, twice the
  variance increase of merging a and b (c = centroids).  The merge height is
  that d (the paper's squared form; scipy's Ward heights are its square root).
* Ties: the pair (i, j), i < j, of smallest distance, then smallest i, then
  smallest j, in the current slot numbering; the merged cluster takes slot
  i and slot j is retired.
* Output in the usual linkage layout: row s = [id_a, id_b, height, size]
  with id_a < id_b, original observations 0..n-1 and the cluster made at
  step s numbered n + s.

Floating point: float64; the squared distances add (x_k - y_k)^2 over the
features in order k = 0, 1, ...; the recurrence is evaluated exactly as
written above, left to right, without fused operations.
"""
from __future__ import annotations

import numpy as np


def squared_distances(X) -> np.ndarray:
    """d_ij = sum_k (X_ik - X_jk)^2, accumulated in feature order."""
    X = np.asarray(X, np.float64)
    n, f = X.shape
    D = np.zeros((n, n))
    for k in range(f):
        t = X[:, k][:, None] - X[:, k][None, :]
        D = D + t * t
    return D


def ward_update(dki, dkj, dij, ni, nj, nk):
    """Lance-Williams distance from cluster k to the union of i and j."""
    return ((ni + nk) * dki + (nj + nk) * dkj - nk * dij) / (ni + nj + nk)


def ward_linkage(X) -> np.ndarray:
    """Ward's agglomeration of the rows of X; (n - 1) x 4 linkage matrix."""
    X = np.asarray(X, np.float64)
    n = X.shape[0]
    D = squared_distances(X)
    active = np.ones(n, bool)
    size = np.ones(n)
    ident = np.arange(n, dtype=np.float64)
    Z = np.zeros((max(n - 1, 0), 4))
    for s in range(n - 1):
        best = (np.inf, n, n)
        for i in range(n):
            if not active[i]:
                continue
            for j in range(i + 1, n):
                if active[j] and D[i, j] < best[0]:
                    best = (D[i, j], i, j)
        dij, i, j = best
        a, b = ident[i], ident[j]
        Z[s] = [min(a, b), max(a, b), dij, size[i] + size[j]]
        for k in range(n):
            if active[k] and k != i and k != j:
                d = ward_update(D[k, i], D[k, j], dij, size[i], size[j], size[k])
                D[k, i] = d
                D[i, k] = d
        size[i] = size[i] + size[j]
        active[j] = False
        ident[i] = n + s
    return Z
