"""The BF16 matrix-core variant of the tiled path (CFSIM_FLAG_MFMA_BF16)
through the C ABI: against the CPU model of its rounding (oracle/bf16_model)
and, reported with a loose bound, against the FP64 oracle; matchings greedy
on the variant's own S; the block cap; the large-pair workload."""
import os

import numpy as np
import pytest

import oracle
from cfgsynth import CFG, Grammar, config_graphs, make_cfg
from tests.parity import check_margin

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "workload2_oracle.npz")
# S of the variant against the model of its rounding: the model sums in FP64,
# the matrix cores in FP32, so an intermediate can round to the neighbouring
# BF16 value (one BF16 unit, 2^-8 relative); the iteration damps such
# perturbations (measured: at most 6.1e-3 on the cases below).  Against FP64
# the error is that of BF16 operands and depends on the pair's spectral gap:
# the model itself is 5.6e-3 to 0.134 from FP64 on the small pairs below and
# ~1e-3 on the large-pair workload; it is reported, not gated, except for a
# sanity bound on the large-pair workload.
MODEL_GATE = 2e-2
LARGE_SANITY_BOUND = 5e-2


@pytest.fixture(scope="module")
def cf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02423_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(cf):
    return cf.Context(0)


def _mat(g):
    return oracle.transition_matrix(g.n, g.src, g.dst, g.count)


def _run(cf, ctx, graphs, pa, pb, **kw):
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, np.asarray(pa, np.int32), np.asarray(pb, np.int32), dtype="f32", want_S=True,
                 want_match=True, path="large", mfma=True, **kw)
    b.run()
    torch.cuda.synchronize()
    return b, b.results(), b.S_list(), b.matches()


def test_mfma_against_model_and_oracle_with_ragged_blocks(cf, ctx):
    rng = np.random.default_rng(71)
    sizes = [(40, 70), (100, 33), (130, 257), (64, 64), (2, 40), (300, 290), (33, 31)]
    graphs = []
    for na, nb in sizes:
        graphs += [make_cfg(na, Grammar(counts="trip"), rng), make_cfg(nb, Grammar(counts="trip"), rng)]
    pa = np.arange(0, 2 * len(sizes), 2)
    b, res, Ss, ms = _run(cf, ctx, graphs, pa, pa + 1)
    worst_model, worst_fp64 = 0.0, 0.0
    for p in range(len(sizes)):
        A, B = _mat(graphs[2 * p]), _mat(graphs[2 * p + 1])
        S = Ss[p].astype(np.float64)
        assert S.shape == (B.shape[0], A.shape[0])
        assert res["status"][p] & (cf.CONVERGED | cf.HIT_MAX_ITER)
        assert abs(np.linalg.norm(S) - 1.0) < 1e-5 and np.all(S >= 0)
        M = oracle.coupled_iteration_bf16(A, B, int(res["iters"][p]), 0.0)[0]
        R = oracle.coupled_iteration(A, B, 200, 1e-12)[0]
        em = np.linalg.norm(S - M) / np.linalg.norm(M)
        ef = np.linalg.norm(S - R) / np.linalg.norm(R)
        worst_model, worst_fp64 = max(worst_model, em), max(worst_fp64, ef)
        own, _ = oracle.greedy_match(S)
        assert np.array_equal(ms[p], own), p
        check_margin(res["margin"][p], S, ms[p], "f32")
        assert abs(res["score"][p] - sum(S[i, j] for i, j in enumerate(ms[p]) if j >= 0)) < 1e-6
    print(f"MFMA BF16: max rel err vs BF16 model {worst_model:.3e}, vs FP64 oracle {worst_fp64:.3e} (reported)")
    assert worst_model <= MODEL_GATE, worst_model


def test_mfma_replay_deterministic(cf, ctx):
    rng = np.random.default_rng(5)
    graphs = [make_cfg(n, Grammar(counts="trip"), rng) for n in (150, 220, 90, 300)]
    b, res, Ss, ms = _run(cf, ctx, graphs, [0, 2], [1, 3])
    r1, S1 = res.tobytes(), b.S.clone()
    for _ in range(2):
        b.res.zero_()
        b.S.zero_()
        b.run()
        torch.cuda.synchronize()
        assert b.results().tobytes() == r1
        assert torch.equal(b.S, S1)


def test_mfma_pair_over_the_block_cap_is_invalid(cf, ctx):
    """4096-node graphs with three random jumps per node hold more nonzero
    32 x 32 blocks than twice the node count: that pair is refused, the other
    pair of the call is served."""
    rng = np.random.default_rng(9)
    n = 4096
    src = np.repeat(np.arange(n, dtype=np.int32), 3)
    dst = rng.integers(0, n, size=3 * n).astype(np.int32)
    dense = CFG(n, src, dst, np.ones(3 * n))
    small = [make_cfg(200, Grammar(counts="trip"), rng), make_cfg(150, Grammar(counts="trip"), rng)]
    b, res, Ss, ms = _run(cf, ctx, [dense, dense] + small, [0, 2], [1, 3], max_iter=4)
    assert res["status"][0] == cf.INVALID_INPUT
    assert res["status"][1] & cf.HIT_MAX_ITER


def test_mfma_workload2_full_launch(cf, ctx):
    """All 64 pairs (512-2048 nodes): every pair served, unit norm, matchings
    greedy on the variant's S; two pairs against stored FP64 oracle samples
    (error reported with the loose bound)."""
    w = config_graphs(2)
    b, res, Ss, ms = _run(cf, ctx, w["graphs"], w["pair_a"], w["pair_b"])
    assert len(res) == 64 and np.all(res["status"] & (cf.CONVERGED | cf.HIT_MAX_ITER))
    gold = np.load(GOLDEN)
    for p in range(64):
        S = Ss[p].astype(np.float64)
        assert abs(np.linalg.norm(S) - 1.0) <= 1e-5
    for p in gold["pairs"]:
        p = int(p)
        S = Ss[p].astype(np.float64)
        own, _ = oracle.greedy_match(S)
        assert np.array_equal(ms[p], own)
        idx, val = gold[f"p{p}_idx"], gold[f"p{p}_val"]
        est = np.sqrt(np.sum((S.reshape(-1)[idx] - val) ** 2) * S.size / idx.size)
        print(f"pair {p}: estimated rel err vs FP64 {est:.3e}")
        assert est <= LARGE_SANITY_BOUND, (p, est)
