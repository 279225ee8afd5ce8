"""Plan tuning of the batched path (step a8): a tune table moves classes of
pairs to larger LDS kernels, the results stay within the oracle gates on the
tuned choices, and the autotuner produces, applies and caches a table."""
import numpy as np
import pytest

from cfgsynth import Grammar, config_graphs, make_cfg
from tests.parity import chain_depth, check_margin, check_matching, check_S, oracle_pair, stop_drift

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_02423_amd as m
    return m


def _check_sample(cf, graphs, pa, pb, res, matches, Ss, sample):
    for p in sample:
        ref = oracle_pair(graphs, int(pa[p]), int(pb[p]))
        er = check_S(Ss[p], ref.S, "f32", max(res["iters"][p], ref.iters), chain_depth(graphs[pa[p]], graphs[pb[p]]),
                     stop_drift(graphs, int(pa[p]), int(pb[p]), res["iters"][p], ref.iters))
        check_margin(res["margin"][p], Ss[p], matches[p], "f32")
        check_matching(Ss[p], matches[p], ref.S, "f32", er)


def test_tune_table_moves_classes_and_keeps_parity(cf):
    ctx = cf.Context(0)
    rng = np.random.default_rng(21)
    sizes = [8, 20, 33, 50, 64, 90, 128]
    graphs = [make_cfg(n, Grammar(counts="trip"), rng) for n in sizes]
    pa, pb = np.triu_indices(len(graphs), k=0)
    pa, pb = pa.astype(np.int32), pb.astype(np.int32)
    gs = cf.pack(ctx, graphs)
    b = cf.Batch(ctx, gs, pa, pb, dtype="f32", want_S=True)
    first = b.buckets()
    ctx.set_tune("f32", [4] * cf.TUNE_CLASSES)   # every class to the largest LDS kernel
    assert ctx.get_tune("f32") == [4] * cf.TUNE_CLASSES
    moved = b.buckets()
    assert np.all(moved >= first)
    assert np.all(moved[first < 5] == 4)          # every LDS pair fits the largest LDS kernel
    b.run()
    torch.cuda.synchronize()
    res, matches, Ss = b.results(), b.matches(), b.S_list()
    _check_sample(cf, graphs, pa, pb, res, matches, Ss, range(len(pa)))
    ctx.set_tune("f32", None)
    assert ctx.get_tune("f32") == [-1] * cf.TUNE_CLASSES
    assert np.array_equal(b.buckets(), first)


def test_autotune_workload1_subset_sets_and_caches_a_table(cf, tmp_path):
    from paper_1707_02423_amd import tune
    ctx = cf.Context(0)
    w = config_graphs(1, scale=40 / 256)
    gs = cf.pack(ctx, w["graphs"])
    rec = tune.autotune(ctx, gs, w["pair_a"], w["pair_b"], "f32", reps=2)
    assert len(rec["table"]) == cf.TUNE_CLASSES and ctx.get_tune("f32") == rec["table"]
    assert all(-1 <= v <= 4 for v in rec["table"])
    for c, info in rec["classes"].items():
        best = min(info["ms_per_pass"].items(), key=lambda kv: kv[1])[0]
        assert str(info["chosen"]) == best or info["chosen"] == -1
    path = tune.save(rec, str(tmp_path))
    ctx2 = cf.Context(0)
    got = tune.load(ctx2, "f32", str(tmp_path))
    assert got is not None and ctx2.get_tune("f32") == rec["table"] and path.endswith("_f32.json")
    # the tuned plan scores within the oracle gates
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_S=True)
    b.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    sample = rng.choice(len(w["pair_a"]), size=24, replace=False)
    _check_sample(cf, w["graphs"], w["pair_a"], w["pair_b"], b.results(), b.matches(), b.S_list(), sample)
