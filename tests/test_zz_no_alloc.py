"""cfsim_score_noalloc (static device scratch, no workspace argument) against
cfsim_score with a caller-owned workspace, through the C ABI: bit for bit
the same outputs, on consecutive calls whose second input is smaller (the
scratch keeps the previous call's contents), on the global-memory kernel
and on the tiled (resized) path; pairs past the scratch are refused before
any HIP call."""
import ctypes

import numpy as np
import pytest

from cfgsynth import Grammar, make_cfg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1707_02423_amd import cfsim
    return cfsim


def _outputs(cfm, gs, a, b, opt, nS, nM):
    dt = torch.float64 if opt.dtype == cfm.F64 else torch.float32
    S = torch.full((nS,), float("nan"), dtype=dt, device="cuda")
    m = torch.full((nM,), -7, dtype=torch.int32, device="cuda")
    r = torch.zeros(cfm.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    return S, m, r


def _run_pair(cfm, ctx, gs, a, b, opt):
    L = cfm.lib()
    A, B = gs.graph(a), gs.graph(b)
    nA, nB = A.n, B.n
    if opt.resize == cfm.RESIZE_BILINEAR:
        nA = nB = max(nA, nB)
    # the existing entry point, with a workspace of its own
    S1, m1, r1 = _outputs(cfm, gs, a, b, opt, nA * nB, nB)
    wsb = L.cfsim_score_workspace_size(ctx.handle, A.n, B.n, ctypes.byref(opt))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    rc = L.cfsim_score(ctx.handle, ctypes.byref(A), ctypes.byref(B), ctypes.byref(opt), S1.data_ptr(),
                       m1.data_ptr(), r1.data_ptr(), ws.data_ptr(), wsb, None)
    assert rc == 0, L.cfsim_last_error()
    # the no-allocation entry point
    S2, m2, r2 = _outputs(cfm, gs, a, b, opt, nA * nB, nB)
    rc = L.cfsim_score_noalloc(ctx.handle, ctypes.byref(A), ctypes.byref(B), ctypes.byref(opt), S2.data_ptr(),
                               m2.data_ptr(), r2.data_ptr(), None)
    assert rc == 0, L.cfsim_last_error()
    torch.cuda.synchronize()
    assert wsb > 0  # the pair uses the scratch
    assert torch.equal(S1, S2)
    assert torch.equal(m1, m2)
    assert torch.equal(r1, r2)
    res = r2.cpu().numpy().view(cfm.RESULT_DTYPE)[0]
    assert res["status"] & (cfm.CONVERGED | cfm.HIT_MAX_ITER)


@pytest.mark.parametrize("dtype,resize,sizes", [
    ("f64", "none", [(300, 250), (210, 140)]),   # global-memory kernel, S in the scratch
    ("f32", "none", [(600, 90), (400, 70)]),
    ("f32", "bilinear", [(40, 120), (20, 60)]),  # tiled path, every iterate in the scratch
])
def test_noalloc_equals_score_on_consecutive_calls(cfm, dtype, resize, sizes):
    ctx = cfm.Context(0)
    rng = np.random.default_rng(len(sizes[0]) * 31 + sizes[0][0])
    graphs = []
    for nA, nB in sizes:
        graphs += [make_cfg(nA, Grammar(counts="trip"), rng), make_cfg(nB, Grammar(counts="trip"), rng)]
    gs = cfm.pack(ctx, graphs)
    opt = cfm.options(dtype, max_iter=60, resize=resize)
    for k in range(len(sizes)):  # second call smaller than the first
        _run_pair(cfm, ctx, gs, 2 * k, 2 * k + 1, opt)


def test_noalloc_refuses_pairs_past_the_scratch(cfm):
    ctx = cfm.Context(0)
    L = cfm.lib()
    rng = np.random.default_rng(5)
    graphs = [make_cfg(1500, Grammar(counts="trip"), rng), make_cfg(1400, Grammar(counts="trip"), rng)]
    gs = cfm.pack(ctx, graphs)
    opt = cfm.options("f64", max_iter=4)
    A, B = gs.graph(0), gs.graph(1)
    assert L.cfsim_score_workspace_size(ctx.handle, A.n, B.n, ctypes.byref(opt)) > cfm.NOALLOC_SCRATCH_BYTES
    r = torch.zeros(cfm.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    rc = L.cfsim_score_noalloc(ctx.handle, ctypes.byref(A), ctypes.byref(B), ctypes.byref(opt), None, None,
                               r.data_ptr(), None)
    assert rc == -6  # CFSIM_E_UNSUPPORTED
    assert b"static scratch" in L.cfsim_last_error()
    torch.cuda.synchronize()
    assert int(r.sum()) == 0  # outputs untouched
