"""Plain FP64 CPU oracle of the optimal-assignment matching.

TEST INFRASTRUCTURE, like the rest of `oracle/`: only `tests/`,
`__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may import
it; it shares no code with the HIP library.

The paper reduces the IsoRank solution to matched node pairs (Section 4.2,
Pairwise Comparison; the IsoRank method it cites extracts matches from the
similarity matrix) without fixing how.  The greedy matching of the hot path
is one reading; this module is the other: the matching of min(n_A, n_B) node
pairs that maximises the total similarity sum S_ij (a linear assignment
problem), with the score being that total.  Unlike the greedy pick, the
optimal total is a Lipschitz function of S (it moves by at most
min(n_A, n_B) max |dS_ij|), so no near-tie contract is needed for the score.

Method: the Hungarian method in its shortest-augmenting-path form (Kuhn,
Munkres; the O(n^2 m) version with row and column potentials).  With the
cost C = -S (transposed when S has more rows than columns, so that
n = rows <= m = columns), rows are inserted one at a time; each insertion
grows a Dijkstra tree over the columns on reduced costs
C[i][j] - u[i] - v[j] until it reaches a free column, shifting the
potentials by the tree's smallest slack at every step, then flips the
matching along the path.  Ties take the smallest column index.

Floating point: float64 throughout; numpy vector operations over the columns
are the library primitives (each entry is computed by the same expression a
scalar loop over j would evaluate); the first index of a minimum is taken.
"""
from __future__ import annotations

import numpy as np


def optimal_assignment(S):
    """Maximum-total matching of min(n_B, n_A) pairs on S (n_B x n_A).

    Returns (match, score): match[i] = j or -1 for the n_B rows and the sum of
    the matched entries taken in ascending row order.  Every entry of S must
    be finite.
    """
    S = np.asarray(S, np.float64)
    nB, nA = S.shape
    if not np.isfinite(S).all():
        raise ValueError("S must be finite")
    transpose = nB > nA
    C = -(S.T if transpose else S)
    n, m = C.shape
    inf = np.inf
    u = np.zeros(n + 1)
    v = np.zeros(m + 1)
    p = np.zeros(m + 1, np.int64)     # p[j]: row (1-based) on column j, 0 = free; column 0 is the root
    way = np.zeros(m + 1, np.int64)   # way[j]: the previous column on the path to j
    for i in range(1, n + 1):
        p[0] = i
        j0 = 0
        minv = np.full(m + 1, inf)
        used = np.zeros(m + 1, bool)
        while True:
            used[j0] = True
            i0 = p[j0]
            free = ~used[1:]
            cur = C[i0 - 1] - u[i0] - v[1:]
            better = free & (cur < minv[1:])
            minv[1:][better] = cur[better]
            way[1:][better] = j0
            cand = np.where(free, minv[1:], inf)
            j1 = int(np.argmin(cand)) + 1
            delta = cand[j1 - 1]
            u[p[used]] += delta
            v[used] -= delta
            minv[~used] -= delta
            j0 = j1
            if p[j0] == 0:
                break
        while j0 != 0:   # flip the matching along the path back to the root
            j1 = way[j0]
            p[j0] = p[j1]
            j0 = j1
    match = np.full(nB, -1, np.int32)
    for j in range(1, m + 1):
        if p[j] != 0:
            if transpose:
                match[j - 1] = p[j] - 1
            else:
                match[p[j] - 1] = j - 1
    score = 0.0
    for i in range(nB):
        if match[i] >= 0:
            score += float(S[i, match[i]])
    return match, score
