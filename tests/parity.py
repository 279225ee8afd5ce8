"""Comparison rules of the HIP results against the FP64 oracle.

* S, element by element: max |S_gpu - S_ref| <= gate * max |S_ref|, with
  gate 1e-10 for FP64 and 1e-5 for FP32 (and the relative Frobenius error
  within the same gate).
* S, entry by entry relative: every product and sum of the iteration has
  non-negative operands, so each computed entry of an update carries at most
  m roundings (m = the longest chain of products and sums behind one entry,
  plus the scale and the store).  A non-negative linear map does not expand
  Hilbert's projective metric (Birkhoff), so after K updates the computed and
  exact iterates are within 2 K m u of each other in that metric, and after
  Frobenius normalisation every entry is within that relative amount:
  |S_gpu - S_ref| / S_ref <= 2 K m u (u = 2^-24 for FP32), and 1e-10 for
  FP64 (whose bound is far below it), on every entry the type holds with
  full precision (S_ref >= 1e-300 or >= 1e-30).  m is taken from the pair's
  degrees: the longest lane list (successors or predecessors of one column
  node) plus the longest row list (successors and predecessors of one row
  node) plus 3.  An FP32 pair may stop at another even step than the FP64
  oracle (its delta is taken from FP32 iterates); the entries then also
  carry the oracle's own change between the two steps, |R_Kgpu - R_Kref|
  from the oracle's iterates, which the per-entry gate allows on top.
* Matching, decided in the kernel's precision: the GPU matching must equal,
  bit for bit, the oracle's greedy applied to the GPU's own S; the kernel's
  margin must equal `relative_margin` of the GPU's own S.
* Matching against the oracle's S: with delta_m = 2 * (the largest per-entry
  relative error of S_gpu), the matchings are identical whenever the oracle
  S has a relative margin above delta_m (a pick's rivals all trail it by a
  relative amount above delta_m); otherwise (a near tie) every GPU pick,
  replayed in the GPU's greedy order on the oracle's S, must be within a
  relative delta_m of the best entry still admissible at that step.
"""
import numpy as np

import oracle

# status bits the oracle also produces (the rest are the kernel's own flags)
BASE_STATUS = oracle.CONVERGED | oracle.HIT_MAX_ITER | oracle.DEGENERATE | oracle.INVALID_INPUT
NEAR_TIE = 16
FP64_FINAL = 32

GATE = {"f64": 1e-10, "f32": 1e-5}
UNIT_ROUNDOFF = {"f64": 2.0 ** -53, "f32": 2.0 ** -24}
DEFAULT_DEPTH = 24  # m for graphs of out-degree <= 2 and in-degree <= 10
ENTRY_FLOOR = {"f64": 1e-300, "f32": 1e-30}
MIN_NORMAL = {"f64": np.finfo(np.float64).tiny, "f32": float(np.finfo(np.float32).tiny)}


def base_status(st):
    return int(st) & BASE_STATUS


def rel_err(S, R):
    S = np.asarray(S, np.float64)
    R = np.asarray(R, np.float64)
    return float(np.linalg.norm(S - R) / np.linalg.norm(R))


def entry_rel_err(S, R, dtype):
    """Largest |S - R| / R over the entries R holds with full precision in dtype."""
    S = np.asarray(S, np.float64)
    R = np.asarray(R, np.float64)
    big = R >= ENTRY_FLOOR[dtype]
    if not big.any():
        return 0.0
    return float(np.max(np.abs(S[big] - R[big]) / R[big]))


def chain_depth(ga, gb):
    """m of the per-entry gate for a pair of graphs (with .n, .src, .dst)."""
    lane, row = 0, 0
    for g in (ga, gb):
        out = np.bincount(np.asarray(g.src, np.int64), minlength=g.n)
        inn = np.bincount(np.asarray(g.dst, np.int64), minlength=g.n)
        lane = max(lane, int(np.max(np.maximum(out, inn))) if g.n else 0)
        row = max(row, int(np.max(out + inn)) if g.n else 0)
    return lane + row + 3


def entry_gate(dtype, iters=200, depth=DEFAULT_DEPTH):
    """Per-entry relative gate after `iters` updates (see the module notes)."""
    if dtype == "f64":
        return 1e-10
    return 2.0 * max(int(iters), 1) * depth * UNIT_ROUNDOFF[dtype]


def stop_drift(graphs, a, b, k_gpu, k_ref):
    """|R_k_gpu - R_k_ref| entry by entry from the oracle's own iterates (0 when
    the update counts agree)."""
    k_gpu, k_ref = int(k_gpu), int(k_ref)
    if k_gpu == k_ref:
        return 0.0
    ga, gb = graphs[a], graphs[b]
    mat = oracle.transition_matrix_sparse if max(ga.n, gb.n) > 128 else oracle.transition_matrix
    A = mat(ga.n, ga.src, ga.dst, ga.count)
    B = mat(gb.n, gb.src, gb.dst, gb.count)
    its = oracle.coupled_iteration(A, B, max(k_gpu, k_ref), 0.0, keep_iterates=True)[5]
    return np.abs(np.asarray(its[k_gpu]) - np.asarray(its[k_ref]))


def check_S(S_gpu, S_ref, dtype, iters=200, depth=DEFAULT_DEPTH, drift=0.0):
    """Element-wise, per-entry relative and Frobenius gates; returns the
    largest per-entry relative error (without the drift allowance)."""
    S = np.asarray(S_gpu, np.float64)
    R = np.asarray(S_ref, np.float64)
    assert S.shape == R.shape, (S.shape, R.shape)
    g = GATE[dtype]
    scale = float(np.max(np.abs(R))) if R.size else 0.0
    dmax = float(np.max(np.abs(S - R))) if R.size else 0.0
    assert dmax <= g * scale, f"element-wise: max |dS| = {dmax:.3e} > {g:.0e} * max|S| = {g * scale:.3e}"
    e = rel_err(S, R)
    assert e <= g, f"relative Frobenius error {e:.3e}"
    er = entry_rel_err(S, R, dtype)
    eg = entry_gate(dtype, iters, depth)
    big = R >= ENTRY_FLOOR[dtype]
    if big.any():
        excess = np.abs(S - R) - np.broadcast_to(drift, R.shape)
        worst = float(np.max(excess[big] / R[big]))
        assert worst <= eg, f"per-entry relative error {worst:.3e} > {eg:.3e} (beyond the stop drift)"
    return er


def _ranks(S):
    flat = np.asarray(S, np.float64).ravel()
    # greedy order: value descending, flat index ascending; NaN last
    v = np.where(np.isnan(flat), -np.inf, flat)
    order = np.lexsort((np.arange(flat.size), np.isnan(flat), -v))
    rank = np.empty(flat.size, np.int64)
    rank[order] = np.arange(flat.size)
    return rank.reshape(S.shape)


def relative_margin(S, match, tiny):
    """Smallest 1 - q / v over the picks v = S[i, match[i]] and their rivals q:
    entries of row i or column match[i] whose other line was unmatched or
    matched later in the greedy order.  A pick below `tiny` counts 0;
    +inf if no pick has a rival."""
    S = np.asarray(S, np.float64)
    nB, nA = S.shape
    R = _ranks(S)
    big = np.iinfo(np.int64).max
    rowpick = np.full(nB, big)
    colpick = np.full(nA, big)
    for i, j in enumerate(match):
        if j >= 0:
            rowpick[i] = R[i, j]
            colpick[j] = R[i, j]
    m = np.inf
    for i, j in enumerate(match):
        if j < 0:
            continue
        v, rk = S[i, j], R[i, j]
        adm_c = colpick > rk
        adm_c[j] = False
        adm_r = rowpick > rk
        adm_r[i] = False
        if not (adm_c.any() or adm_r.any()):
            continue
        if not v >= tiny:
            m = min(m, 0.0)
            continue
        q = -np.inf
        if adm_c.any():
            q = max(q, np.nanmax(S[i, adm_c]))
        if adm_r.any():
            q = max(q, np.nanmax(S[adm_r, j]))
        m = min(m, 1.0 - q / v)
    return m


def check_margin(res_margin, S_gpu, match_gpu, dtype):
    """The kernel's margin equals the margin of its own matching on its own S."""
    want = relative_margin(np.asarray(S_gpu, np.float64), match_gpu, MIN_NORMAL[dtype])
    got = float(res_margin)
    if np.isinf(want):
        assert np.isinf(got) and got > 0, (got, want)
    else:
        assert abs(got - want) <= 1e-15 * max(1.0, abs(want)), (got, want)


def check_matching(S_gpu, match_gpu, S_ref, dtype="f32", entry_err=None):
    """Returns "exact" or "near-tie"; raises AssertionError on a violation."""
    S_gpu64 = np.asarray(S_gpu, np.float64)
    own, _ = oracle.greedy_match(S_gpu64)
    assert np.array_equal(np.asarray(match_gpu), own), "GPU matching differs from greedy on the GPU's own S"
    if entry_err is None:
        entry_err = entry_rel_err(S_gpu64, S_ref, dtype)
    dm = max(2.0 * entry_err, 1e-12)
    ref_match, _ = oracle.greedy_match(S_ref)
    # picks below the full-precision floor count as ties
    if relative_margin(S_ref, ref_match, ENTRY_FLOOR[dtype]) > dm:
        assert np.array_equal(np.asarray(match_gpu), ref_match), "matching differs on a well-separated pair"
        return "exact"
    certify_near_tie(S_gpu64, match_gpu, S_ref, dm, ENTRY_FLOOR[dtype])
    return "near-tie"


def certify_near_tie(S_gpu, match_gpu, S_ref, dm, floor):
    """Replays the GPU's picks in its greedy order on the oracle's S: each must
    be within a relative dm (or below `floor`) of the best admissible entry."""
    S_gpu = np.asarray(S_gpu, np.float64)
    nB, nA = S_gpu.shape
    picks = [(i, int(j)) for i, j in enumerate(match_gpu) if j >= 0]
    picks.sort(key=lambda e: (-S_gpu[e], e[0] * nA + e[1]))
    avail = np.ones_like(S_ref, bool)
    for (i, j) in picks:
        best = np.where(avail, S_ref, -np.inf).max()
        ok = S_ref[i, j] >= best * (1.0 - dm) or best < floor
        assert ok, f"near-tie pick ({i}, {j}) = {S_ref[i, j]:.6e} trails the best admissible {best:.6e}"
        avail[i, :] = False
        avail[:, j] = False


def oracle_pair(graphs, a, b, max_iter=200, tol=1e-12, resize="none"):
    ga, gb = graphs[a], graphs[b]
    A = oracle.transition_matrix(ga.n, ga.src, ga.dst, ga.count)
    B = oracle.transition_matrix(gb.n, gb.src, gb.dst, gb.count)
    return oracle.score_pair(A, B, max_iter, tol, resize)
