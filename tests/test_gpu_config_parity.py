"""Oracle parity at the full shapes of the query-vs-database and backward
workloads: a seeded sample of the 65,536 query pairs (including pairs that
take the global-memory kernel) with the top-16 of that sample, the reverse
mode at 16-256 nodes against the oracle's reverse mode, and central finite
differences of the FP64 oracle on 32 sampled pairs of the backward workload."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from cfgsynth import config_graphs
from tests.parity import chain_depth, check_matching, check_S, stop_drift

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02423_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(cf):
    return cf.Context(0)


def _mat(g, sparse=False):
    if sparse:
        return oracle.transition_matrix_sparse(g.n, g.src, g.dst, g.count)
    return oracle.transition_matrix(g.n, g.src, g.dst, g.count)


def test_query_database_full_size_sampled(cf, ctx):
    """The 200-node query against all 65,536 database graphs (FP32, one
    batched call): 64 seeded pairs against the oracle, 16 of them with more
    than 128 database nodes (global-memory kernel), and the top-16 of the
    sample from the GPU scores against the top-16 of the oracle scores."""
    w = config_graphs(4)
    graphs, pa, pb = w["graphs"], w["pair_a"], w["pair_b"]
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, pa, pb, dtype="f32", want_match=True, want_S=True)
    b.run()
    torch.cuda.synchronize()
    res = b.results()
    assert len(res) == 65536 and np.all(res["status"] != cf.INVALID_INPUT)
    nb = np.array([graphs[g].n for g in pb])
    rng = np.random.default_rng(4242)
    big = rng.choice(np.flatnonzero(nb > 128), size=16, replace=False)
    rest = rng.choice(np.flatnonzero(nb <= 128), size=48, replace=False)
    sample = np.concatenate([big, rest])
    bk = b.buckets()
    assert np.all(bk[big] == 5), "pairs over 128 database nodes take the global-memory kernel"
    ref_scores = np.empty(len(sample))
    for k, p in enumerate(sample):
        ga, gb = graphs[pa[p]], graphs[pb[p]]
        ref = oracle.score_pair(_mat(ga, True), _mat(gb, True), 200, 1e-12)
        ref_S = np.asarray(ref.S)
        o, nA, nB = int(b.S_off_h[p]), int(b.nA[p]), int(b.nB[p])
        S = b.S[o:o + nA * nB].cpu().numpy().reshape(nB, nA)
        er = check_S(S, ref_S, "f32", max(res["iters"][p], ref.iters), chain_depth(ga, gb),
                     stop_drift(graphs, int(pa[p]), int(pb[p]), res["iters"][p], ref.iters))
        m = b.match[int(b.match_off_h[p]):int(b.match_off_h[p]) + nB].cpu().numpy()
        check_matching(S, m, ref_S, "f32", er)
        ref_scores[k] = ref.score
        assert abs(res["score"][p] - ref.score) <= 1e-4 * max(1.0, ref.score)
    gpu_scores = torch.as_tensor(res["score"][sample], device="cuda")
    gi, _ = cf.topk(ctx, gpu_scores, 16)
    gi = gi.cpu().numpy()
    ri, rv = oracle.topk(ref_scores, 16)
    for r in range(16):
        if gi[r] != ri[r]:  # only where the oracle scores are within the FP32 score error
            assert abs(ref_scores[gi[r]] - rv[r]) <= 1e-4 * max(1.0, abs(rv[r])), (r, gi[r], ri[r])


def _to_input_order(gs, g_csr, graphs, which):
    out = {}
    for g in which:
        G = graphs[g]
        e0 = int(gs.edge_off[g])
        order = np.lexsort((np.arange(G.nnz), G.dst, G.src))
        v = np.zeros(G.nnz)
        v[order] = g_csr[e0:e0 + G.nnz]
        out[g] = v
    return out


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-9), ("f32", 5e-4)])
def test_backward_workload3_sizes_vs_oracle_reverse_mode(cf, ctx, dtype, tol):
    """Pairs of the backward workload at its extremes (the largest area, a
    16-node side, a mixed pair), K as the forward found it (<= 200),
    against the oracle's reverse mode."""
    w = config_graphs(3)
    graphs, pa, pb = w["graphs"], w["pair_a"], w["pair_b"]
    area = np.array([graphs[a].n * graphs[c].n for a, c in zip(pa, pb)])
    small = np.array([min(graphs[a].n, graphs[c].n) for a, c in zip(pa, pb)])
    pick = [int(np.argmax(area)), int(np.argmin(small)), int(np.argsort(area)[len(area) // 2])]
    sel_a, sel_b = pa[pick], pb[pick]
    used = sorted(set(sel_a.tolist()) | set(sel_b.tolist()))
    sub = [graphs[g] for g in used]
    ia = np.array([used.index(g) for g in sel_a], np.int32)
    ib = np.array([used.index(g) for g in sel_b], np.int32)
    gs = cf.pack(ctx, sub)
    b = cf.Batch(ctx, gs, ia, ib, dtype=dtype, want_match=True)
    b.run()
    torch.cuda.synchronize()
    res, matches = b.results(), b.matches()
    gsc = np.array([1.0, 0.75, 1.25])
    grad = torch.zeros(gs.total_edges, dtype=torch.float64, device="cuda")
    st = cf.backward(b, torch.as_tensor(gsc), grad, checkpoint_every=8)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    got = _to_input_order(gs, grad.cpu().numpy(), sub, range(len(sub)))
    for p in range(3):
        ga, gb = sub[ia[p]], sub[ib[p]]
        dA, dB = oracle.backward(_mat(ga), _mat(gb), int(res["iters"][p]), matches[p])
        for g, G, dX in ((ia[p], ga, dA), (ib[p], gb, dB)):
            ref = gsc[p] * oracle.edge_gradients(dX, G.src, G.dst)
            scale = max(np.abs(ref).max(), 1e-300)
            err = np.abs(got[g] - ref).max() / scale
            assert err <= tol, (p, G.n, err)


def test_backward_finite_differences_32_sampled_pairs(cf, ctx):
    """Central differences (h = 1e-6, FP64 oracle, K and the matching held at
    the forward's) on 32 seeded pairs of the backward workload, 3 edges of each
    graph, against the FP32 reverse mode of the whole 1,024-pair batch with
    grad_score = 1 on the sampled pairs (whose graphs are not shared) and 0
    elsewhere."""
    w = config_graphs(3)
    graphs, pa, pb = w["graphs"], w["pair_a"], w["pair_b"]
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, pa, pb, dtype="f32", want_match=True)
    b.run()
    torch.cuda.synchronize()
    res, matches = b.results(), b.matches()
    rng = np.random.default_rng(33)
    sample = rng.choice(len(pa), size=32, replace=False)
    touched = np.concatenate([pa[sample], pb[sample]])
    assert len(set(touched.tolist())) == 64, "sampled pairs must not share graphs"
    gsc = np.zeros(len(pa))
    gsc[sample] = 1.0
    grad = torch.zeros(gs.total_edges, dtype=torch.float64, device="cuda")
    st = cf.backward(b, torch.as_tensor(gsc), grad, checkpoint_every=8)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    got = _to_input_order(gs, grad.cpu().numpy(), graphs, touched.tolist())
    h = 1e-6
    worst = 0.0
    for p in sample:
        K, m = int(res["iters"][p]), matches[p]
        ga, gb = graphs[pa[p]], graphs[pb[p]]
        A, B = _mat(ga, True), _mat(gb, True)
        for which, g, G, X in (("A", pa[p], ga, A), ("B", pb[p], gb, B)):
            for e in rng.choice(G.nnz, size=min(3, G.nnz), replace=False):
                u, v = int(G.src[e]), int(G.dst[e])
                if X[u, v] == 0.0:
                    continue  # a zero-count jump: the packer keeps it, the derivative is still defined
                f = []
                for sgn in (1, -1):
                    Xh = X.copy().tolil()
                    Xh[u, v] += sgn * h
                    Xh = sp.csr_matrix(Xh)
                    S = oracle.coupled_iteration(Xh, B, K, -1.0)[0] if which == "A" else \
                        oracle.coupled_iteration(A, Xh, K, -1.0)[0]
                    S = np.asarray(S)
                    f.append(sum(S[i, j] for i, j in enumerate(m) if j >= 0))
                fd = (f[0] - f[1]) / (2 * h)
                worst = max(worst, abs(got[g][e] - fd) / max(1.0, abs(fd)))
    assert worst < 5e-4, worst
