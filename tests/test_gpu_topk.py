"""Top-k on the device against the oracle's ordering (bit-exact: indices)."""
import numpy as np
import pytest

import oracle

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


@pytest.mark.parametrize("n,k", [(1, 1), (5, 3), (7, 10), (4096, 16), (4097, 16), (65536, 16), (100000, 64),
                                 (9000, 1024)])
def test_topk_matches_oracle_with_ties_and_nan(cf, ctx, n, k):
    rng = np.random.default_rng(n + k)
    s = np.round(rng.random(n), 2)          # many exact ties
    s[rng.random(n) < 0.01] = np.nan          # invalid pairs
    idx, val = cf.topk(ctx, torch.as_tensor(s, device="cuda"), k)
    ref_i, ref_v = oracle.topk(s, k)
    kk = min(k, n)
    assert idx.cpu().numpy()[:kk].tolist() == ref_i[:kk].tolist()
    np.testing.assert_array_equal(val.cpu().numpy()[:kk], ref_v[:kk])
    if k > n:
        assert np.all(idx.cpu().numpy()[n:] == -1)


def test_topk_on_batch_results(cf, ctx):
    from cfgsynth import config_graphs
    w = config_graphs(4, scale=600 / 65536)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=False)
    b.run()
    idx, val = b.topk(16)
    torch.cuda.synchronize()
    res = b.results()
    ref_i, ref_v = oracle.topk(res["score"], 16)
    assert idx.cpu().numpy().tolist() == ref_i.tolist()
    np.testing.assert_array_equal(val.cpu().numpy(), ref_v)
