"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before any HIP call (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1707_02423_amd import cfsim as cf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfsim.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfsim_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = cf.lib()
    names = _declared()
    assert "cfsim_score" in names and "cfsim_score_batch" in names and "cfsim_pack" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(cf.SIGNATURES), set(names) - set(cf.SIGNATURES)


def test_version_and_empty_error():
    L = cf.lib()
    assert L.cfsim_version().startswith(b"cfsim")


def _graph(n=3, nnz=2):
    # pointers are never dereferenced: every case below fails validation first
    return cf.Graph(n, nnz, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000)


def _call_score(A, B, opt, res=0x1000, ws=0x1000, ws_bytes=1 << 30):
    L = cf.lib()
    return L.cfsim_score(None, ctypes.byref(A) if A is not None else None, ctypes.byref(B) if B is not None else None,
                         ctypes.byref(opt) if opt is not None else None, None, None, res, ws, ws_bytes, None)


@pytest.mark.parametrize("case,code,text", [
    ("null_opt", -1, "options"),
    ("bad_dtype", -1, "dtype"),
    ("max_iter0", -1, "max_iter"),
    ("nan_tol", -1, "tol"),
    ("neg_tol", -1, "tol"),
    ("flags", -1, "flags"),
    ("fp64_final_f64", -1, "FP32 calls only"),
    ("nan_tie_tol", -1, "tie_tol"),
    ("neg_tie_tol", -1, "tie_tol"),
    ("bad_resize", -1, "resize"),
    ("n0", -2, "n must be"),
    ("nnz_neg", -2, "nnz"),
    ("null_edges", -1, "edge array"),
    ("null_graph", -1, "NULL"),
    ("null_res", -1, "res"),
    ("null_ctx", -1, "context"),
    ("small_ws", -5, "workspace"),
])
def test_score_validation(case, code, text):
    A, B = _graph(), _graph(4, 3)
    opt = cf.options("f64")
    res = 0x1000
    if case == "null_opt":
        opt = None
    elif case == "bad_dtype":
        opt.dtype = 7
    elif case == "max_iter0":
        opt.max_iter = 0
    elif case == "nan_tol":
        opt.tol = float("nan")
    elif case == "neg_tol":
        opt.tol = -1.0
    elif case == "flags":
        opt.flags = 4
    elif case == "fp64_final_f64":
        opt.flags = 1
    elif case == "nan_tie_tol":
        opt.tie_tol = float("nan")
    elif case == "neg_tie_tol":
        opt.tie_tol = -1e-3
    elif case == "bad_resize":
        opt.resize = 5
    elif case == "n0":
        A.n = 0
    elif case == "nnz_neg":
        B.nnz = -1
    elif case == "null_edges":
        A.col = None
    elif case == "null_graph":
        A = None
    elif case == "null_res":
        res = None
    ws_bytes = 16 if case == "small_ws" else 1 << 30
    got = _call_score(A, B, opt, res, ws_bytes=ws_bytes)
    assert got == code
    assert text in cf.lib().cfsim_last_error().decode()


def test_score_workspace_size():
    L = cf.lib()
    opt = cf.options("f32")
    assert L.cfsim_score_workspace_size(None, 12, 16, ctypes.byref(opt)) >= 2 * 12 * 16 * 4
    assert L.cfsim_score_workspace_size(None, 0, 16, ctypes.byref(opt)) == 0


def test_score_too_large_pair_is_unsupported():
    A, B = _graph(3000, 4000), _graph(3000, 4000)
    assert _call_score(A, B, cf.options("f32")) == -6
    assert "do not fit" in cf.lib().cfsim_last_error().decode()


def _set(**kw):
    s = cf.GraphSetC(4, 10, 30, 40, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


@pytest.mark.parametrize("kw,n_pairs,ws,code,text", [
    (dict(n_graphs=0), 5, 1 << 20, -2, "n_graphs"),
    (dict(max_nodes=0), 5, 1 << 20, -2, "max_nodes"),
    (dict(total_nodes=2), 5, 1 << 20, -2, "total_nodes"),
    (dict(node_off=None), 5, 1 << 20, -1, "offset"),
    (dict(w=None), 5, 1 << 20, -1, "edge array"),
    ({}, -1, 1 << 20, -1, "n_pairs"),
    ({}, 5, 16, -5, "workspace"),
    ({}, 5, 1 << 40, -1, "context"),
])
def test_batch_validation(kw, n_pairs, ws, code, text):
    L = cf.lib()
    s = _set(**kw)
    opt = cf.options("f32")
    got = L.cfsim_score_batch(None, ctypes.byref(s), 0x1000, 0x1000, n_pairs, ctypes.byref(opt), 0x1000, None, None,
                              None, None, 0x1000, ws, None)
    assert got == code
    assert text in L.cfsim_last_error().decode()


def test_batch_requires_paired_optional_outputs():
    L = cf.lib()
    s = _set()
    opt = cf.options("f32")
    got = L.cfsim_score_batch(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), 0x1000, 0x1000, None,
                              None, None, 0x1000, 1 << 20, None)
    assert got == -1 and "match_off" in L.cfsim_last_error().decode()


def test_batch_workspace_size_grows_with_pairs():
    L = cf.lib()
    s = _set()
    opt = cf.options("f32")
    a = L.cfsim_batch_workspace_size(None, ctypes.byref(s), 10, ctypes.byref(opt))
    b = L.cfsim_batch_workspace_size(None, ctypes.byref(s), 100000, ctypes.byref(opt))
    assert 0 < a < b and b >= 400000


def test_pack_validation():
    L = cf.lib()
    P = 0x1000
    assert L.cfsim_pack(None, -1, 0, 0, P, P, P, P, P, P, P, P, P, P, P, P, P, 1 << 20, None) == -1
    assert L.cfsim_pack(None, 2, 5, 4, None, P, P, P, P, P, P, P, P, P, P, P, P, 1 << 20, None) == -1
    assert L.cfsim_pack(None, 2, 5, 4, P, P, P, P, P, P, P, P, P, P, P, P, P, 4, None) == -5
    assert L.cfsim_pack(None, 2, 5, 4, P, P, P, P, P, P, P, P, P, P, P, P, P, 1 << 20, None) == -1
    assert "context" in L.cfsim_last_error().decode()
    assert L.cfsim_pack_workspace_size(2, 5, 4) >= 5 * 4 + 2 * 4 * 4


def test_context_create_rejects_null_out():
    assert cf.lib().cfsim_context_create(None, 0) == -1


def test_topk_validation():
    L = cf.lib()
    P = 0x1000
    assert L.cfsim_topk(None, P, 0, 1, 4, P, P, P, 1 << 20, None) == -1
    assert L.cfsim_topk(None, P, 10, 0, 4, P, P, P, 1 << 20, None) == -1
    assert L.cfsim_topk(None, P, 10, 1, 0, P, P, P, 1 << 20, None) == -1
    assert L.cfsim_topk(None, P, 10, 1, 2000, P, P, P, 1 << 20, None) == -1
    assert L.cfsim_topk(None, P, 10, 1, 4, P, P, P, 1, None) == -5
    assert L.cfsim_topk(None, P, 10, 1, 4, P, P, P, 1 << 20, None) == -1
    assert "context" in L.cfsim_last_error().decode()
    assert L.cfsim_topk_workspace_size(65536, 16) >= 16 * 16 * 16


def test_bucket_and_timing_validation():
    L = cf.lib()
    s = _set()
    opt = cf.options("f32")
    assert L.cfsim_batch_buckets(None, ctypes.byref(s), 0x1000, 0x1000, -1, ctypes.byref(opt), 0x1000, None) == -1
    assert L.cfsim_batch_buckets(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), None, None) == -1
    assert "bucket" in L.cfsim_last_error().decode()
    assert L.cfsim_batch_buckets(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), 0x1000, None) == -1
    assert "context" in L.cfsim_last_error().decode()
    assert L.cfsim_context_set_timing(None, 1) == -1
    assert L.cfsim_batch_timings(None, None) == -1


def test_bucket_kernel_names():
    assert cf.NUM_BUCKETS == 7
    names = [cf.bucket_kernel(b, "f32") for b in range(cf.NUM_BUCKETS)]
    assert names[0].startswith("pair_lds_kernel<float, 64,") and names[5] == "pair_global_kernel<float>"
    assert names[6] == "" and cf.bucket_kernel(-1) == "" and cf.bucket_kernel(0, 7) == ""
    assert all("double" in cf.bucket_kernel(b, "f64") for b in range(6))
    assert len(set(names[:6])) == 6


@pytest.mark.parametrize("kw,n_pairs,ws,opt_kw,code,text", [
    ({}, -1, 1 << 40, {}, -1, "n_pairs"),
    (dict(max_nodes=9000), 5, 1 << 40, {}, -6, "8192"),
    ({}, 5, 1 << 40, dict(max_iter=5000), -6, "4096"),
    ({}, 5, 16, {}, -5, "workspace"),
    ({}, 5, 1 << 40, {}, -1, "context"),
])
def test_large_validation(kw, n_pairs, ws, opt_kw, code, text):
    L = cf.lib()
    s = _set(**kw)
    opt = cf.options("f32", **opt_kw)
    got = L.cfsim_score_large(None, ctypes.byref(s), 0x1000, 0x1000, n_pairs, ctypes.byref(opt), 0x1000, None, None,
                              None, None, 0x1000, ws, None)
    assert got == code
    assert text in L.cfsim_last_error().decode()


def test_large_workspace_size():
    L = cf.lib()
    s = _set(max_nodes=2048)
    opt = cf.options("f32")
    one = L.cfsim_large_workspace_size(None, ctypes.byref(s), 1, ctypes.byref(opt))
    assert one >= 4 * 2048 * 2048 * 4
    assert L.cfsim_large_workspace_size(None, ctypes.byref(s), 64, ctypes.byref(opt)) >= 64 * 4 * 2048 * 2048 * 4
    assert L.cfsim_large_workspace_size(None, ctypes.byref(_set(max_nodes=9000)), 1, ctypes.byref(opt)) == 0


def test_resize_limits_and_unsupported_calls():
    L = cf.lib()
    opt = cf.options("f32", resize="bilinear")
    s = _set(max_nodes=9000)
    assert L.cfsim_score_batch(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), 0x1000, None, None,
                               None, None, 0x1000, 1 << 40, None) == -6
    assert "8192" in L.cfsim_last_error().decode()
    assert L.cfsim_batch_workspace_size(None, ctypes.byref(s), 5, ctypes.byref(opt)) == 0
    s = _set()
    # resized calls have buckets (LDS kernels in their resized mode, the rest on the tiled path)
    assert L.cfsim_batch_buckets(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), 0x1000, None) == -1
    assert "context" in L.cfsim_last_error().decode()
    assert L.cfsim_score_backward(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), 0x1000, 0x1000,
                                  0x1000, 0x1000, 0x1000, None, 8, None, None, 0x1000, 1 << 40, None) == -6
    opt_long = cf.options("f32", max_iter=5000, resize="bilinear")
    A, B = _graph(), _graph(4, 3)
    assert _call_score(A, B, opt_long) == -6


def test_resize_workspace_sizes():
    L = cf.lib()
    opt = cf.options("f32", resize="bilinear")
    # plain: one pair, six n_M^2 slots
    assert L.cfsim_score_workspace_size(None, 12, 16, ctypes.byref(opt)) >= 6 * 16 * 16 * 4
    s = _set(max_nodes=128)
    assert L.cfsim_batch_workspace_size(None, ctypes.byref(s), 100, ctypes.byref(opt)) >= 100 * 6 * 128 * 128 * 4


def test_result_and_options_layout():
    """The ctypes mirrors have the sizes of the C structs (40 and 32 bytes)."""
    assert cf.RESULT_BYTES == 40 and cf.RESULT_STRIDE == 5
    assert ctypes.sizeof(cf.Options) == 32
    assert [n for n, _ in cf.Options._fields_] == ["dtype", "max_iter", "tol", "resize", "flags", "tie_tol"]
    assert cf.RESULT_DTYPE.names == ("score", "nu", "delta", "margin", "iters", "status")


def test_fp64_final_refused_where_it_does_not_apply():
    L = cf.lib()
    s = _set()
    opt = cf.options("f32", resize="bilinear", fp64_final=True)
    assert L.cfsim_score_batch(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), 0x1000, None, None,
                               None, None, 0x1000, 1 << 40, None) == -6
    assert "FP64_FINAL" in L.cfsim_last_error().decode()
    opt = cf.options("f32", fp64_final=True)
    assert L.cfsim_score_large(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), 0x1000, None, None,
                               None, None, 0x1000, 1 << 40, None) == -6
    assert L.cfsim_score_backward(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), 0x1000, 0x1000,
                                  0x1000, 0x1000, 0x1000, None, 8, None, None, 0x1000, 1 << 40, None) == -6
    # the FP64 pass needs FP64-sized global-kernel slots
    plain = cf.options("f32")
    a = L.cfsim_batch_workspace_size(None, ctypes.byref(s), 10, ctypes.byref(plain))
    b = L.cfsim_batch_workspace_size(None, ctypes.byref(s), 10, ctypes.byref(opt))
    assert b > a
    assert (L.cfsim_score_workspace_size(None, 12, 16, ctypes.byref(opt)) >=
            2 * L.cfsim_score_workspace_size(None, 12, 16, ctypes.byref(plain)) - 256)


class _G:
    def __init__(self, n, src, dst, count):
        self.n, self.src, self.dst, self.count = n, src, dst, count


@pytest.mark.parametrize("graphs,code,text", [
    ([_G(3, [0, 1], [1, 2], [1.0, 2.0]), _G(2, [0], [1], [0.0])], 0, ""),
    ([_G(3, [0, 1], [1, 3], [1.0, 2.0])], -2, "graph 0, jump 1: endpoint (1, 3) outside [0, 3)"),
    ([_G(2, [0], [1], [1.0]), _G(2, [-1], [1], [1.0])], -2, "graph 1, jump 0"),
    ([_G(2, [0, 1], [1, 0], [1.0, float("nan")])], -3, "graph 0, jump 1: count is not finite"),
    ([_G(2, [0], [1], [float("inf")])], -3, "not finite"),
    ([_G(4, [0, 1, 2], [1, 2, 3], [1.0, -0.5, 2.0])], -4, "graph 0, jump 1: negative count"),
    ([_G(1, [], [], [])], 0, ""),
])
def test_check_jumps(graphs, code, text):
    """Host validation returns the documented status and names the first bad jump."""
    if code == 0:
        cf.check_jumps(graphs)
        return
    with pytest.raises(cf.CfsimError) as e:
        cf.check_jumps(graphs)
    assert e.value.code == code and text in str(e.value)


def test_check_jumps_offsets():
    L = cf.lib()
    import numpy as np
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    no = np.array([0, 2, 2], np.int64)     # second graph has no node
    eo = np.array([0, 0, 0], np.int64)
    z = np.zeros(1, np.int32)
    assert L.cfsim_check_jumps(2, p(no), p(eo), p(z), p(z), p(np.zeros(1))) == -2
    assert "node_off must increase" in L.cfsim_last_error().decode()
    no = np.array([0, 2, 4], np.int64)
    eo = np.array([0, 3, 1], np.int64)     # decreasing edge offsets
    assert L.cfsim_check_jumps(2, p(no), p(eo), p(z), p(z), p(np.zeros(1))) == -2
    assert "edge_off decreases" in L.cfsim_last_error().decode()
    assert L.cfsim_check_jumps(1, None, p(eo), None, None, None) == -1


def test_score_noalloc_validation():
    """The no-allocation entry point checks its arguments, then its scratch
    bound, on the host before any HIP call."""
    L = cf.lib()
    A, B = _graph(), _graph(4, 3)
    opt = cf.options("f64")
    call = lambda ctx, A, B, opt, res: L.cfsim_score_noalloc(
        ctx, ctypes.byref(A) if A is not None else None, ctypes.byref(B), ctypes.byref(opt) if opt else None,
        None, None, res, None)
    assert call(None, None, B, opt, 0x1000) == -1 and "NULL" in L.cfsim_last_error().decode()
    assert call(None, A, B, None, 0x1000) == -1 and "options" in L.cfsim_last_error().decode()
    assert call(None, A, B, opt, None) == -1 and "res" in L.cfsim_last_error().decode()
    assert call(None, A, B, opt, 0x1000) == -1 and "context" in L.cfsim_last_error().decode()
    # past the scratch: FP64 2 * n_A * n_B * 8 bytes > 16 MiB
    big_a, big_b = _graph(1500, 2000), _graph(1400, 1900)
    assert L.cfsim_score_workspace_size(None, 1500, 1400, ctypes.byref(opt)) > cf.NOALLOC_SCRATCH_BYTES
    got = L.cfsim_score_noalloc(ctypes.c_void_p(0x1000), ctypes.byref(big_a), ctypes.byref(big_b),
                                ctypes.byref(opt), None, None, 0x1000, None)
    assert got == -6 and "static scratch" in L.cfsim_last_error().decode()


def test_tune_class_and_table_validation():
    """Tune classes are half octaves of n_A * n_B; the table calls check
    their arguments on the host."""
    L = cf.lib()
    assert L.cfsim_tune_class(1, 1) == 0
    assert L.cfsim_tune_class(8, 16) == 14
    assert L.cfsim_tune_class(128, 128) == 28
    assert L.cfsim_tune_class(100, 7) == int(2 * np.log2(700))
    assert L.cfsim_tune_class(60000, 60000) == cf.TUNE_CLASSES - 1
    arr = (ctypes.c_int32 * cf.TUNE_CLASSES)(*([-1] * cf.TUNE_CLASSES))
    assert L.cfsim_context_set_tune(None, cf.F32, arr, cf.TUNE_CLASSES) == -1
    assert "context" in L.cfsim_last_error().decode()
    assert L.cfsim_context_get_tune(None, cf.F32, arr, cf.TUNE_CLASSES) == -1


def test_forward_checkpoint_arguments_checked_on_the_host():
    L = cf.lib()
    s = _set()
    opt = cf.options("f32")
    call = lambda ck, off, every, o=opt: L.cfsim_score_batch_ckpt(
        None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(o), 0x1000, None, None, None, None, ck, off, every,
        0x1000, 1 << 40, None)
    assert call(0x1000, 0x1000, 0) == -1 and "checkpoint_every" in L.cfsim_last_error().decode()
    assert call(None, 0x1000, 8) == -1 and "ckpt" in L.cfsim_last_error().decode()
    assert call(0x1000, 0x1000, 8, cf.options("f32", resize="bilinear")) == -6
    assert call(0x1000, 0x1000, 8, cf.options("f32", fp64_final=True)) == -6
    assert call(0x1000, 0x1000, 8) == -1 and "context" in L.cfsim_last_error().decode()
    # the backward takes both checkpoint arrays or neither
    assert L.cfsim_score_backward(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), 0x1000, 0x1000,
                                  0x1000, 0x1000, 0x1000, None, 8, 0x1000, None, 0x1000, 1 << 40, None) == -1
    assert "ckpt" in L.cfsim_last_error().decode()


@pytest.mark.parametrize("kw,n_pairs,p,ws,code,text", [
    (dict(n_graphs=0), 5, 3.0, 1 << 20, -2, "n_graphs"),
    ({}, -1, 3.0, 1 << 20, -1, "n_pairs"),
    ({}, 5, 0.5, 1 << 20, -1, "Minkowski"),
    ({}, 5, float("inf"), 1 << 20, -1, "Minkowski"),
    ({}, 5, float("nan"), 1 << 20, -1, "Minkowski"),
    (dict(max_nodes=40000), 5, 3.0, 1 << 20, -6, "max_nodes"),
    ({}, 5, 3.0, 1 << 20, -1, "context"),
])
def test_distances_validation(kw, n_pairs, p, ws, code, text):
    L = cf.lib()
    s = _set(**kw)
    assert L.cfsim_distances(None, ctypes.byref(s), 0x1000, 0x1000, n_pairs, p, 0x1000, 0x1000, ws, None) == code
    assert text in L.cfsim_last_error().decode()


def test_distances_null_buffers_and_workspace():
    L = cf.lib()
    s = _set()
    P = 0x1000
    assert L.cfsim_distances(P, ctypes.byref(s), None, P, 5, 3.0, P, P, 1 << 20, None) == -1
    assert L.cfsim_distances(P, ctypes.byref(s), P, P, 5, 3.0, None, P, 1 << 20, None) == -1
    need = L.cfsim_distances_workspace_size(ctypes.byref(s), 5)
    assert need > 0
    assert L.cfsim_distances(P, ctypes.byref(s), P, P, 5, 3.0, P, P, need - 1, None) == -5
    assert "workspace" in L.cfsim_last_error().decode()
    # No pair: nothing to do, no workspace needed and no HIP call.
    assert L.cfsim_distances(P, ctypes.byref(s), None, None, 0, 3.0, None, None, 0, None) == 0


def test_distances_workspace_bound_covers_every_size():
    L = cf.lib()
    # Chunk partials: at most 64 chunks of six doubles per pair.
    small = L.cfsim_distances_workspace_size(ctypes.byref(_set(max_nodes=8)), 1000)
    large = L.cfsim_distances_workspace_size(ctypes.byref(_set(max_nodes=2048)), 1000)
    assert small >= 1001 * 8 + 1000 * 48 and large >= 1001 * 8 + 1000 * 64 * 48
    assert L.cfsim_distances_workspace_size(ctypes.byref(_set(max_nodes=40000)), 10) == 0


@pytest.mark.parametrize("alpha,prior,prior_off,opt_kw,code,text", [
    (-0.1, None, None, {}, -1, "alpha"),
    (1.0, None, None, {}, -1, "alpha"),
    (float("nan"), None, None, {}, -1, "alpha"),
    (0.85, 0x1000, None, {}, -1, "prior"),
    (0.85, None, 0x1000, {}, -1, "prior"),
    (0.85, None, None, dict(resize="bilinear"), -6, "unscaled"),
    (0.85, None, None, dict(mfma=True), -6, ""),
    (0.85, None, None, {}, -1, "context"),
])
def test_damped_arguments_checked_on_the_host(alpha, prior, prior_off, opt_kw, code, text):
    L = cf.lib()
    s = _set()
    opt = cf.options("f32", **opt_kw)
    got = L.cfsim_score_damped(None, ctypes.byref(s), 0x1000, 0x1000, 5, ctypes.byref(opt), alpha, prior, prior_off,
                               0x1000, None, None, None, None, 0x1000, 1 << 40, None)
    assert got == code
    assert text in L.cfsim_last_error().decode()


@pytest.mark.parametrize("dtype,n_pairs,max_dim,ptrs,code,text", [
    (5, 3, 16, {}, -1, "dtype"),
    (0, -1, 16, {}, -1, "n_pairs"),
    (0, 3, 0, {}, -1, "max_dim"),
    (1, 3, 5000, {}, -6, "max_dim"),
    (0, 3, 16, dict(S=None), -1, "NULL"),
    (0, 3, 16, dict(score=None), -1, "NULL"),
    (0, 3, 16, dict(match_off=None), -1, "match"),
    (0, 3, 16, {}, -1, "context"),
])
def test_assign_arguments_checked_on_the_host(dtype, n_pairs, max_dim, ptrs, code, text):
    L = cf.lib()
    P = 0x1000
    a = dict(S=P, S_off=P, n_rows=P, n_cols=P, match=P, match_off=P, score=P)
    a.update(ptrs)
    got = L.cfsim_assign(None, dtype, a["S"], a["S_off"], a["n_rows"], a["n_cols"], n_pairs, max_dim, a["match"],
                         a["match_off"], a["score"], None)
    assert got == code
    assert text in L.cfsim_last_error().decode()
    # no matrix: nothing to do and no HIP call
    assert L.cfsim_assign(P, 0, None, None, None, None, 0, 16, None, None, None, None) == 0


def test_ward_arguments_checked_on_the_host():
    L = cf.lib()
    P = 0x1000
    assert L.cfsim_ward_workspace_size(100) >= 100 * 100 * 8
    assert L.cfsim_ward_workspace_size(0) == 0 and L.cfsim_ward_workspace_size(5000) == 0
    cases = [
        ((P, P, 0, 3, P, P, 1 << 20, None), -1, "n_obs"),
        ((P, P, 10, 0, P, P, 1 << 20, None), -1, "n_feat"),
        ((P, P, 5000, 3, P, P, 1 << 40, None), -6, "observations"),
        ((P, None, 10, 3, P, P, 1 << 20, None), -1, "NULL"),
        ((P, P, 10, 3, None, P, 1 << 20, None), -1, "NULL"),
        ((P, P, 10, 3, P, P, 16, None), -5, "workspace"),
        ((None, P, 10, 3, P, P, 1 << 20, None), -1, "context"),
    ]
    for args, code, text in cases:
        assert L.cfsim_ward(*args) == code, args
        assert text in L.cfsim_last_error().decode()
    # one observation: no merge, no HIP call
    assert L.cfsim_ward(P, P, 1, 3, None, P, 1 << 20, None) == 0
