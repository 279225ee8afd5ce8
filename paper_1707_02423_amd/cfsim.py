"""Python binding of libcfsim (argument marshalling only).

Every step of the similarity runs in the HIP kernels of libcfsim.so; this
module only moves arguments: it lays out device buffers with PyTorch (memory
and streams), passes raw pointers through ctypes, and reads results back.
There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcfsim.so")

F64, F32 = 0, 1
RESIZE_NONE, RESIZE_BILINEAR = 0, 1
CONVERGED, HIT_MAX_ITER, DEGENERATE, INVALID_INPUT, NEAR_TIE, FP64_FINAL = 1, 2, 4, 8, 16, 32
FLAG_FP64_FINAL = 1
FLAG_MFMA_BF16 = 2
NUM_BUCKETS = 7  # batch buckets: 0-4 LDS kernels, 5 global-memory kernel, 6 invalid pairs
PACK_BAD_INDEX, PACK_NONFINITE, PACK_NEGATIVE = 1, 2, 4
NOALLOC_SCRATCH_BYTES = 16 << 20  # CFSIM_NOALLOC_SCRATCH_BYTES
TUNE_CLASSES = 32  # CFSIM_TUNE_CLASSES

STATUS_NAMES = {0: "CFSIM_OK", -1: "CFSIM_E_INVALID_ARG", -2: "CFSIM_E_BAD_GRAPH", -3: "CFSIM_E_NONFINITE",
                -4: "CFSIM_E_NEGWEIGHT", -5: "CFSIM_E_WORKSPACE", -6: "CFSIM_E_UNSUPPORTED", -7: "CFSIM_E_HIP"}

RESULT_DTYPE = np.dtype([("score", "<f8"), ("nu", "<f8"), ("delta", "<f8"), ("margin", "<f8"), ("iters", "<i4"),
                         ("status", "<u4")])
RESULT_BYTES = RESULT_DTYPE.itemsize        # 40: sizeof(cfsim_pair_result)
RESULT_STRIDE = RESULT_BYTES // 8           # doubles per result (score at 0)


class CfsimError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
                ("resize", ctypes.c_int32), ("flags", ctypes.c_uint32), ("tie_tol", ctypes.c_double)]


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("col_ptr", ctypes.c_void_p),
                ("row", ctypes.c_void_p), ("eid", ctypes.c_void_p)]


class GraphSetC(ctypes.Structure):
    _fields_ = [("n_graphs", ctypes.c_int32), ("max_nodes", ctypes.c_int32), ("total_nodes", ctypes.c_int64),
                ("total_edges", ctypes.c_int64), ("node_off", ctypes.c_void_p), ("edge_off", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("col_ptr", ctypes.c_void_p), ("row", ctypes.c_void_p), ("eid", ctypes.c_void_p)]


_LIB = None
_P = ctypes.c_void_p
_SZ = ctypes.c_size_t
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64

# name -> (restype, argtypes); must mirror include/cfsim.h
SIGNATURES = {
    "cfsim_last_error": (ctypes.c_char_p, []),
    "cfsim_version": (ctypes.c_char_p, []),
    "cfsim_context_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int]),
    "cfsim_context_destroy": (None, [_P]),
    "cfsim_check_jumps": (ctypes.c_int, [_I32, _P, _P, _P, _P, _P]),
    "cfsim_pack_workspace_size": (_SZ, [_I32, _I64, _I64]),
    "cfsim_pack": (ctypes.c_int, [_P, _I32, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ,
                                  _P]),
    "cfsim_score_workspace_size": (_SZ, [_P, _I32, _I32, ctypes.POINTER(Options)]),
    "cfsim_score": (ctypes.c_int, [_P, ctypes.POINTER(Graph), ctypes.POINTER(Graph), ctypes.POINTER(Options), _P, _P,
                                   _P, _P, _SZ, _P]),
    "cfsim_score_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(Graph), ctypes.POINTER(Graph), ctypes.POINTER(Options),
                                           _P, _P, _P, _P]),
    "cfsim_batch_workspace_size": (_SZ, [_P, ctypes.POINTER(GraphSetC), _I64, ctypes.POINTER(Options)]),
    "cfsim_score_batch": (ctypes.c_int, [_P, ctypes.POINTER(GraphSetC), _P, _P, _I64, ctypes.POINTER(Options), _P,
                                         _P, _P, _P, _P, _P, _SZ, _P]),
    "cfsim_backward_workspace_size": (_SZ, [_P, ctypes.POINTER(GraphSetC), _I64, ctypes.POINTER(Options), _I32]),
    "cfsim_score_batch_ckpt": (ctypes.c_int, [_P, ctypes.POINTER(GraphSetC), _P, _P, _I64,
                                              ctypes.POINTER(Options), _P, _P, _P, _P, _P, _P, _P, _I32, _P, _SZ,
                                              _P]),
    "cfsim_score_backward": (ctypes.c_int, [_P, ctypes.POINTER(GraphSetC), _P, _P, _I64, ctypes.POINTER(Options),
                                            _P, _P, _P, _P, _P, _P, _I32, _P, _P, _P, _SZ, _P]),
    "cfsim_large_workspace_size": (_SZ, [_P, ctypes.POINTER(GraphSetC), _I64, ctypes.POINTER(Options)]),
    "cfsim_score_large": (ctypes.c_int, [_P, ctypes.POINTER(GraphSetC), _P, _P, _I64, ctypes.POINTER(Options), _P,
                                         _P, _P, _P, _P, _P, _SZ, _P]),
    "cfsim_batch_buckets": (ctypes.c_int, [_P, ctypes.POINTER(GraphSetC), _P, _P, _I64, ctypes.POINTER(Options),
                                           _P, _P]),
    "cfsim_bucket_kernel": (ctypes.c_char_p, [_I32, _I32]),
    "cfsim_context_set_timing": (ctypes.c_int, [_P, _I32]),
    "cfsim_batch_timings": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float)]),
    "cfsim_tune_class": (_I32, [_I32, _I32]),
    "cfsim_context_set_tune": (ctypes.c_int, [_P, _I32, _P, _I32]),
    "cfsim_context_get_tune": (ctypes.c_int, [_P, _I32, _P, _I32]),
    "cfsim_topk_workspace_size": (_SZ, [_I64, _I32]),
    "cfsim_topk": (ctypes.c_int, [_P, _P, _I64, _I64, _I32, _P, _P, _P, _SZ, _P]),
    "cfsim_score_damped": (ctypes.c_int, [_P, ctypes.POINTER(GraphSetC), _P, _P, _I64, ctypes.POINTER(Options),
                                          ctypes.c_double, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "cfsim_assign": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _I64, _I32, _P, _P, _P, _P]),
    "cfsim_ward_workspace_size": (_SZ, [_I32]),
    "cfsim_ward": (ctypes.c_int, [_P, _P, _I32, _I32, _P, _P, _SZ, _P]),
    "cfsim_distances_workspace_size": (_SZ, [ctypes.POINTER(GraphSetC), _I64]),
    "cfsim_distances": (ctypes.c_int, [_P, ctypes.POINTER(GraphSetC), _P, _P, _I64, ctypes.c_double, _P, _P, _SZ,
                                       _P]),
}


def lib():
    """The loaded libcfsim.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1707_02423_amd/build.py "
                               "(or __graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _check(code: int):
    if code != 0:
        raise CfsimError(code, lib().cfsim_last_error().decode())


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def options(dtype="f64", max_iter=200, tol=1e-12, resize="none", tie_tol=0.0, fp64_final=False,
            mfma=False) -> Options:
    d = {"f64": F64, "f32": F32}[dtype] if isinstance(dtype, str) else int(dtype)
    r = {"none": RESIZE_NONE, "bilinear": RESIZE_BILINEAR}[resize] if isinstance(resize, str) else int(resize)
    flags = (FLAG_FP64_FINAL if fp64_final else 0) | (FLAG_MFMA_BF16 if mfma else 0)
    return Options(dtype=d, max_iter=int(max_iter), tol=float(tol), resize=r, flags=flags, tie_tol=float(tie_tol))


class Context:
    """A libcfsim context bound to one HIP device."""

    def __init__(self, device: int = 0):
        h = _P()
        _check(lib().cfsim_context_create(ctypes.byref(h), int(device)))
        self.handle = h
        self.device = int(device)

    def set_timing(self, on: bool):
        """Eager batched launches with an event pair around each bucket kernel."""
        _check(lib().cfsim_context_set_timing(self.handle, 1 if on else 0))

    def set_tune(self, dtype: str, table):
        """Batch plan tune table of `dtype` (TUNE_CLASSES entries, -1 = default; None resets)."""
        d = {"f64": F64, "f32": F32}[dtype]
        if table is None:
            _check(lib().cfsim_context_set_tune(self.handle, d, None, TUNE_CLASSES))
            return
        arr = (ctypes.c_int32 * TUNE_CLASSES)(*[int(x) for x in table])
        _check(lib().cfsim_context_set_tune(self.handle, d, arr, TUNE_CLASSES))

    def get_tune(self, dtype: str) -> list:
        d = {"f64": F64, "f32": F32}[dtype]
        arr = (ctypes.c_int32 * TUNE_CLASSES)()
        _check(lib().cfsim_context_get_tune(self.handle, d, arr, TUNE_CLASSES))
        return list(arr)

    def batch_timings(self) -> np.ndarray:
        """Milliseconds of each bucket kernel of the last timed batch call (waits for it)."""
        ms = (ctypes.c_float * NUM_BUCKETS)()
        _check(lib().cfsim_batch_timings(self.handle, ms))
        return np.array(ms[:], dtype=np.float64)

    def close(self):
        if getattr(self, "handle", None):
            lib().cfsim_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class GraphSet:
    """A packed, device-resident set of graphs (output of `pack`)."""
    n_graphs: int
    max_nodes: int
    node_off: np.ndarray   # host copy, int64 [G+1]
    edge_off: np.ndarray   # host copy, int64 [G+1]
    d_node_off: torch.Tensor
    d_edge_off: torch.Tensor
    row_ptr: torch.Tensor
    col: torch.Tensor
    w: torch.Tensor
    col_ptr: torch.Tensor
    row: torch.Tensor
    eid: torch.Tensor

    @property
    def total_nodes(self) -> int:
        return int(self.node_off[-1])

    @property
    def total_edges(self) -> int:
        return int(self.edge_off[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.node_off)

    def c_struct(self, w: torch.Tensor | None = None) -> GraphSetC:
        w = self.w if w is None else w
        return GraphSetC(self.n_graphs, self.max_nodes, self.total_nodes, self.total_edges,
                         _ptr(self.d_node_off), _ptr(self.d_edge_off), _ptr(self.row_ptr), _ptr(self.col), _ptr(w),
                         _ptr(self.col_ptr), _ptr(self.row), _ptr(self.eid))

    def graph(self, g: int) -> Graph:
        """A cfsim_graph view of graph g (pointers into the packed arrays)."""
        n0, n1 = int(self.node_off[g]), int(self.node_off[g + 1])
        e0, e1 = int(self.edge_off[g]), int(self.edge_off[g + 1])
        i4, f8 = 4, 8
        return Graph(n1 - n0, e1 - e0,
                     self.row_ptr.data_ptr() + (n0 + g) * i4, self.col.data_ptr() + e0 * i4,
                     self.w.data_ptr() + e0 * f8, self.col_ptr.data_ptr() + (n0 + g) * i4,
                     self.row.data_ptr() + e0 * i4, self.eid.data_ptr() + e0 * i4)

    def host_csr(self, g: int):
        """(row_ptr, col, w) of graph g copied to the host."""
        n0, n1 = int(self.node_off[g]), int(self.node_off[g + 1])
        e0, e1 = int(self.edge_off[g]), int(self.edge_off[g + 1])
        return (self.row_ptr[n0 + g:n1 + g + 1].cpu().numpy(), self.col[e0:e1].cpu().numpy(),
                self.w[e0:e1].cpu().numpy())


def concat_coo(graphs):
    """Concatenate per-graph jump lists (objects with n, src, dst, count)."""
    ns = np.array([g.n for g in graphs], np.int64)
    ms = np.array([len(g.src) for g in graphs], np.int64)
    node_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    edge_off = np.concatenate([[0], np.cumsum(ms)]).astype(np.int64)
    src = np.concatenate([np.asarray(g.src, np.int32) for g in graphs]) if graphs else np.zeros(0, np.int32)
    dst = np.concatenate([np.asarray(g.dst, np.int32) for g in graphs]) if graphs else np.zeros(0, np.int32)
    cnt = np.concatenate([np.asarray(g.count, np.float64) for g in graphs]) if graphs else np.zeros(0)
    return node_off, edge_off, src, dst, cnt


def check_jumps(graphs):
    """Host validation of jump lists (cfsim_check_jumps): raises CfsimError
    (E_BAD_GRAPH, E_NONFINITE, E_NEGWEIGHT) naming the first bad jump."""
    node_off, edge_off, src, dst, cnt = concat_coo(graphs)
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    cnt = np.ascontiguousarray(cnt, np.float64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().cfsim_check_jumps(len(graphs), p(node_off), p(edge_off), p(src), p(dst), p(cnt)))


def pack(ctx: Context, graphs, device=None, stream=None, check=True) -> GraphSet:
    """Step a1 on the device: jump lists with counts -> CSR/CSC transition matrices.
    With check=True the lists are validated on the host first (check_jumps)."""
    dev = torch.device("cuda", ctx.device) if device is None else torch.device(device)
    if check and graphs:
        check_jumps(graphs)
    node_off, edge_off, src, dst, cnt = concat_coo(graphs)
    G = len(graphs)
    N, E = int(node_off[-1]), int(edge_off[-1])
    t = lambda a, dt: torch.as_tensor(a, dtype=dt).to(dev)
    d_node_off, d_edge_off = t(node_off, torch.int64), t(edge_off, torch.int64)
    d_src, d_dst, d_cnt = t(src, torch.int32), t(dst, torch.int32), t(cnt, torch.float64)
    rp = torch.empty(N + G, dtype=torch.int32, device=dev)
    cp = torch.empty(N + G, dtype=torch.int32, device=dev)
    col = torch.empty(max(E, 1), dtype=torch.int32, device=dev)
    row = torch.empty(max(E, 1), dtype=torch.int32, device=dev)
    eid = torch.empty(max(E, 1), dtype=torch.int32, device=dev)
    w = torch.empty(max(E, 1), dtype=torch.float64, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    ws_bytes = lib().cfsim_pack_workspace_size(G, N, E)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    _check(lib().cfsim_pack(ctx.handle, G, N, E, _ptr(d_node_off), _ptr(d_edge_off), _ptr(d_src), _ptr(d_dst),
                            _ptr(d_cnt), _ptr(rp), _ptr(col), _ptr(w), _ptr(cp), _ptr(row), _ptr(eid), _ptr(err),
                            _ptr(ws), ws_bytes, _stream(stream)))
    if check:
        flags = int(err.item())
        if flags:
            raise ValueError(f"cfsim_pack flagged the input (bits {flags:#x}: 1 = bad node id, "
                             "2 = non-finite count, 4 = negative count)")
    max_nodes = int(np.diff(node_off).max()) if G else 1
    return GraphSet(G, max(max_nodes, 1), node_off, edge_off, d_node_off, d_edge_off, rp, col, w, cp, row, eid)


def _torch_dtype(opt: Options):
    return torch.float64 if opt.dtype == F64 else torch.float32


def score(ctx: Context, gs: GraphSet, a: int, b: int, dtype="f64", max_iter=200, tol=1e-12, resize="none",
          want_S=True, stream=None, sync=True, tie_tol=0.0, fp64_final=False):
    """Plain path, one pair: A = graph a, B = graph b of the set."""
    opt = options(dtype, max_iter, tol, resize, tie_tol, fp64_final)
    A, B = gs.graph(a), gs.graph(b)
    dev = gs.w.device
    nA, nB = A.n, B.n
    if opt.resize == RESIZE_BILINEAR:  # S is n_M x n_M, n_M = max(n_A, n_B)
        nA = nB = max(A.n, B.n)
    S = torch.empty(nB * nA, dtype=_torch_dtype(opt), device=dev) if want_S else None
    match = torch.empty(nB, dtype=torch.int32, device=dev)
    res = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=dev)
    ws_bytes = lib().cfsim_score_workspace_size(ctx.handle, A.n, B.n, ctypes.byref(opt))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    _check(lib().cfsim_score(ctx.handle, ctypes.byref(A), ctypes.byref(B), ctypes.byref(opt), _ptr(S), _ptr(match),
                             _ptr(res), _ptr(ws), ws_bytes, _stream(stream)))
    out = dict(S=S, match=match, res=res)
    if sync:
        return finish_single(out, nB, nA)
    return out


def finish_single(out, nB, nA):
    r = out["res"].cpu().numpy().view(RESULT_DTYPE)[0]
    d = {k: r[k].item() for k in RESULT_DTYPE.names}
    d["match"] = out["match"].cpu().numpy()
    if out["S"] is not None:
        d["S"] = out["S"].cpu().numpy().reshape(nB, nA)
    return d


class Batch:
    """Pre-allocated buffers for repeated batched scoring of a fixed pair list.

    `run()` enqueues one batched call (a replay of the cached HIP graph after
    the first call) on the current stream and returns immediately.
    """

    def __init__(self, ctx: Context, gs: GraphSet, pair_a, pair_b, dtype="f32", max_iter=200, tol=1e-12,
                 resize="none", want_match=True, want_S=False, w: torch.Tensor | None = None, path="batch",
                 tie_tol=0.0, fp64_final=False, mfma=False, checkpoint_every=0, alpha=None, prior=None):
        if path not in ("batch", "large", "damped"):
            raise ValueError("path must be 'batch' (cfsim_score_batch), 'large' (cfsim_score_large) "
                             "or 'damped' (cfsim_score_damped)")
        if (path == "damped") != (alpha is not None):
            raise ValueError("alpha is given exactly for the damped path")
        self.path = path
        self.alpha = None if alpha is None else float(alpha)
        self.ctx, self.gs = ctx, gs
        self.opt = options(dtype, max_iter, tol, resize, tie_tol, fp64_final, mfma)
        dev = gs.w.device
        self.pair_a_h = np.asarray(pair_a, np.int32)
        self.pair_b_h = np.asarray(pair_b, np.int32)
        self.n_pairs = int(self.pair_a_h.shape[0])
        self.pair_a = torch.as_tensor(self.pair_a_h).to(dev)
        self.pair_b = torch.as_tensor(self.pair_b_h).to(dev)
        self.res = torch.empty(max(self.n_pairs, 1) * RESULT_BYTES, dtype=torch.uint8, device=dev)
        sizes = gs.sizes().astype(np.int64)

        def size_of(idx):  # 0 for ids outside the set (the kernel marks those pairs invalid)
            ok = (idx >= 0) & (idx < gs.n_graphs)
            return np.where(ok, sizes[np.clip(idx, 0, gs.n_graphs - 1)], 0).astype(np.int64)
        nA, nB = size_of(self.pair_a_h), size_of(self.pair_b_h)
        if self.opt.resize == RESIZE_BILINEAR:  # S is n_M x n_M, n_M = max(n_A, n_B)
            nM = np.where((nA > 0) & (nB > 0), np.maximum(nA, nB), 0)
            nA, nB = nM, nM
        self.nA, self.nB = nA, nB
        self.match = self.match_off = self.S = self.S_off = None
        if want_match:
            off = np.concatenate([[0], np.cumsum(nB)]).astype(np.int64)
            self.match_off_h = off[:-1]
            self.match_off = torch.as_tensor(self.match_off_h).to(dev)
            self.match = torch.empty(max(int(off[-1]), 1), dtype=torch.int32, device=dev)
        if want_S:
            off = np.concatenate([[0], np.cumsum(nA * nB)]).astype(np.int64)
            self.S_off_h = off[:-1]
            self.S_off = torch.as_tensor(self.S_off_h).to(dev)
            self.S = torch.empty(max(int(off[-1]), 1), dtype=_torch_dtype(self.opt), device=dev)
        # forward checkpoints for the reverse mode: S_k every checkpoint_every
        # updates (max_iter // checkpoint_every iterates of n_A n_B per pair)
        self.checkpoint_every = int(checkpoint_every)
        self.ckpt = self.ckpt_off = None
        if self.checkpoint_every > 0:
            if path != "batch":
                raise ValueError("forward checkpoints are taken on the batched path")
            per = (int(max_iter) // self.checkpoint_every) * nA * nB
            off = np.concatenate([[0], np.cumsum(per)]).astype(np.int64)
            self.ckpt_off = torch.as_tensor(off[:-1]).to(dev)
            self.ckpt = torch.empty(max(int(off[-1]), 1), dtype=_torch_dtype(self.opt), device=dev)
        # damped path: the caller's priors, one n_B x n_A FP64 array per pair
        # (None: uniform), packed with their element offsets
        self.prior = self.prior_off = None
        if prior is not None:
            if path != "damped":
                raise ValueError("a prior is taken by the damped path only")
            if len(prior) != self.n_pairs:
                raise ValueError("one prior per pair")
            flat = [np.asarray(x, np.float64).reshape(-1) for x in prior]
            for x, a, b in zip(flat, nA, nB):
                if x.size != a * b:
                    raise ValueError("prior p must hold n_B x n_A entries")
            off = np.concatenate([[0], np.cumsum([x.size for x in flat])]).astype(np.int64)
            self.prior_off = torch.as_tensor(off[:-1]).to(dev)
            self.prior = torch.as_tensor(np.concatenate(flat) if flat else np.zeros(1)).to(dev)
        self.w = w
        self.set_c = gs.c_struct(w)
        size_fn = lib().cfsim_large_workspace_size if path == "large" else lib().cfsim_batch_workspace_size
        self.ws_bytes = size_fn(ctx.handle, ctypes.byref(self.set_c), self.n_pairs, ctypes.byref(self.opt))
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)

    def run(self, stream=None):
        if self.ckpt is not None:
            _check(lib().cfsim_score_batch_ckpt(
                self.ctx.handle, ctypes.byref(self.set_c), _ptr(self.pair_a), _ptr(self.pair_b), self.n_pairs,
                ctypes.byref(self.opt), _ptr(self.res), _ptr(self.match), _ptr(self.match_off), _ptr(self.S),
                _ptr(self.S_off), _ptr(self.ckpt), _ptr(self.ckpt_off), self.checkpoint_every, _ptr(self.ws),
                self.ws_bytes, _stream(stream)))
            return
        if self.path == "damped":
            _check(lib().cfsim_score_damped(
                self.ctx.handle, ctypes.byref(self.set_c), _ptr(self.pair_a), _ptr(self.pair_b), self.n_pairs,
                ctypes.byref(self.opt), self.alpha, _ptr(self.prior), _ptr(self.prior_off), _ptr(self.res),
                _ptr(self.match), _ptr(self.match_off), _ptr(self.S), _ptr(self.S_off), _ptr(self.ws),
                self.ws_bytes, _stream(stream)))
            return
        fn = lib().cfsim_score_batch if self.path == "batch" else lib().cfsim_score_large
        _check(fn(self.ctx.handle, ctypes.byref(self.set_c), _ptr(self.pair_a),
                  _ptr(self.pair_b), self.n_pairs, ctypes.byref(self.opt), _ptr(self.res),
                  _ptr(self.match), _ptr(self.match_off), _ptr(self.S), _ptr(self.S_off),
                  _ptr(self.ws), self.ws_bytes, _stream(stream)))

    def buckets(self, stream=None) -> np.ndarray:
        """The bucket (kernel) the plan gives each pair (see bucket_kernel)."""
        out = torch.empty(max(self.n_pairs, 1), dtype=torch.int32, device=self.pair_a.device)
        _check(lib().cfsim_batch_buckets(self.ctx.handle, ctypes.byref(self.set_c), _ptr(self.pair_a),
                                         _ptr(self.pair_b), self.n_pairs, ctypes.byref(self.opt), _ptr(out),
                                         _stream(stream)))
        return out[: self.n_pairs].cpu().numpy()

    def topk(self, k: int, stream=None):
        """Top-k of this batch's scores, on the device (call after run())."""
        scores = self.res[: self.n_pairs * RESULT_BYTES].view(torch.float64)
        return topk(self.ctx, scores, k, stride=RESULT_STRIDE, n=self.n_pairs, stream=stream)

    def results(self) -> np.ndarray:
        return self.res[: self.n_pairs * RESULT_BYTES].cpu().numpy().view(RESULT_DTYPE)

    def matches(self):
        m = self.match.cpu().numpy()
        return [m[o:o + n] for o, n in zip(self.match_off_h, self.nB)]

    def assign(self, stream=None):
        """Optimal-assignment matching of every pair's S (call after run() of a
        batch built with want_S=True): (matches, scores), device tensors laid
        out like the greedy ones (match_off) and one FP64 score per pair."""
        if self.S is None:
            raise ValueError("the assignment reads S: build the Batch with want_S=True")
        dev = self.S.device
        off = np.concatenate([[0], np.cumsum(self.nB)]).astype(np.int64)
        match = torch.empty(max(int(off[-1]), 1), dtype=torch.int32, device=dev)
        match_off = torch.as_tensor(off[:-1]).to(dev)
        scores = torch.empty(max(self.n_pairs, 1), dtype=torch.float64, device=dev)
        nr = torch.as_tensor(self.nB.astype(np.int32)).to(dev)
        nc = torch.as_tensor(self.nA.astype(np.int32)).to(dev)
        max_dim = int(max(int(self.nA.max(initial=1)), int(self.nB.max(initial=1)), 1))
        _check(lib().cfsim_assign(self.ctx.handle, self.opt.dtype, _ptr(self.S), _ptr(self.S_off), _ptr(nr),
                                  _ptr(nc), self.n_pairs, max_dim, _ptr(match), _ptr(match_off), _ptr(scores),
                                  _stream(stream)))
        self._assign_keep = (nr, nc, match_off)  # alive until the stream has used them
        return match, scores[: self.n_pairs]

    def S_list(self):
        S = self.S.cpu().numpy()
        return [S[o:o + a * b].reshape(b, a) for o, a, b in zip(self.S_off_h, self.nA, self.nB)]


def bucket_kernel(bucket: int, dtype="f32") -> str:
    """Name of the kernel that serves a batch bucket ("" for the invalid bucket)."""
    d = {"f64": F64, "f32": F32}[dtype] if isinstance(dtype, str) else int(dtype)
    return lib().cfsim_bucket_kernel(int(bucket), d).decode()


def topk(ctx: Context, scores: torch.Tensor, k: int, stride: int = 1, n: int | None = None, stream=None):
    """Step a11 on the device: indices and values of the k best scores
    (ties to the lower index, NaN ranks last).  `scores` is a float64 device
    tensor read with `stride` (RESULT_STRIDE reads the score field of a result array)."""
    n = int(scores.numel() // stride) if n is None else int(n)
    dev = scores.device
    idx = torch.empty(k, dtype=torch.int32, device=dev)
    val = torch.empty(k, dtype=torch.float64, device=dev)
    ws_bytes = lib().cfsim_topk_workspace_size(n, k)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    _check(lib().cfsim_topk(ctx.handle, _ptr(scores), n, stride, k, _ptr(idx), _ptr(val), _ptr(ws), ws_bytes,
                            _stream(stream)))
    return idx, val


NUM_DISTANCES = 5
DISTANCE_NAMES = ("euclidean", "manhattan", "minkowski", "jaccard", "cosine")


def distances(ctx: Context, gs: GraphSet, pair_a, pair_b, p: float = 3.0, stream=None) -> torch.Tensor:
    """Table 1's five elementwise distances of every pair (cfsim_distances):
    a float64 device tensor [n_pairs, 5] in the order of DISTANCE_NAMES,
    computed on the two transition matrices at their common size.  The pair
    indices may be host arrays or int32 device tensors (used in place)."""
    dev = gs.row_ptr.device

    def on_device(x):
        if isinstance(x, torch.Tensor):
            return x.to(device=dev, dtype=torch.int32).contiguous()
        return torch.as_tensor(np.asarray(x, np.int32), device=dev)
    pa, pb = on_device(pair_a), on_device(pair_b)
    n = int(pa.numel())
    out = torch.empty((n, NUM_DISTANCES), dtype=torch.float64, device=dev)
    set_c = gs.c_struct()
    L = lib()
    ws_bytes = L.cfsim_distances_workspace_size(ctypes.byref(set_c), n)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    _check(L.cfsim_distances(ctx.handle, ctypes.byref(set_c), _ptr(pa), _ptr(pb), n, float(p), _ptr(out), _ptr(ws),
                             ws_bytes, _stream(stream)))
    return out


def backward(batch: "Batch", grad_score: torch.Tensor, grad_w: torch.Tensor, checkpoint_every: int = 8,
             stream=None) -> torch.Tensor:
    """Step a10: adds d(sum_p grad_score[p] score_p)/dw to grad_w (FP64, CSR
    order of the set) for the pairs of a batch that has run.  Returns the
    per-pair status (0, or INVALID_INPUT for skipped pairs).  A batch built
    with the same checkpoint_every hands its forward checkpoints over; else
    the forward is recomputed."""
    if batch.match is None:
        raise ValueError("the backward needs the forward's matchings: build the Batch with want_match=True")
    dev = batch.gs.w.device
    gsc = grad_score.to(device=dev, dtype=torch.float64).contiguous()
    status = torch.empty(max(batch.n_pairs, 1), dtype=torch.int32, device=dev)
    L = lib()
    ws_bytes = L.cfsim_backward_workspace_size(batch.ctx.handle, ctypes.byref(batch.set_c), batch.n_pairs,
                                               ctypes.byref(batch.opt), int(checkpoint_every))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    use_ck = batch.ckpt is not None and batch.checkpoint_every == int(checkpoint_every)
    ck, ck_off = (batch.ckpt, batch.ckpt_off) if use_ck else (None, None)
    _check(L.cfsim_score_backward(batch.ctx.handle, ctypes.byref(batch.set_c), _ptr(batch.pair_a),
                                  _ptr(batch.pair_b), batch.n_pairs, ctypes.byref(batch.opt), _ptr(batch.res),
                                  _ptr(batch.match), _ptr(batch.match_off), _ptr(gsc), _ptr(grad_w), _ptr(status),
                                  int(checkpoint_every), _ptr(ck), _ptr(ck_off), _ptr(ws), ws_bytes,
                                  _stream(stream)))
    return status[: batch.n_pairs]


class CfsimScore(torch.autograd.Function):
    """scores = CfsimScore.apply(w, ctx, gs, pair_a, pair_b, dtype, max_iter, tol, checkpoint_every)

    w is the packed edge-weight tensor (FP64, CSR order of `gs`, e.g. gs.w or
    a tensor computed from counts with torch); the result is the FP64 score of
    every pair.  backward returns d(loss)/dw through the hand-written adjoint
    kernel (matching and update count held fixed)."""

    @staticmethod
    def forward(ctx_, w, cfctx, gs, pair_a, pair_b, dtype="f32", max_iter=200, tol=1e-12, checkpoint_every=8):
        w = w.detach().contiguous()
        b = Batch(cfctx, gs, pair_a, pair_b, dtype=dtype, max_iter=max_iter, tol=tol, want_match=True, w=w,
                  checkpoint_every=checkpoint_every)
        b.run()
        ctx_.batch = b
        ctx_.w = w
        ctx_.checkpoint_every = checkpoint_every
        return b.res[: b.n_pairs * RESULT_BYTES].view(torch.float64)[0::RESULT_STRIDE].clone()

    @staticmethod
    def backward(ctx_, grad_scores):
        grad_w = torch.zeros_like(ctx_.w, dtype=torch.float64)
        backward(ctx_.batch, grad_scores, grad_w, ctx_.checkpoint_every)
        return grad_w, None, None, None, None, None, None, None, None


def score_batch(ctx, gs, pair_a, pair_b, dtype="f32", max_iter=200, tol=1e-12, resize="none", want_match=True,
                want_S=False, path="batch", tie_tol=0.0, fp64_final=False):
    """Batched (or large-pair) path: run once, synchronise, return (results, matches, S list)."""
    b = Batch(ctx, gs, pair_a, pair_b, dtype, max_iter, tol, resize, want_match, want_S, path=path,
              tie_tol=tie_tol, fp64_final=fp64_final)
    b.run()
    torch.cuda.synchronize()
    return b.results(), (b.matches() if want_match else None), (b.S_list() if want_S else None)


def score_damped(ctx, gs, pair_a, pair_b, alpha=0.85, prior=None, dtype="f32", max_iter=200, tol=1e-12,
                 want_match=True, want_S=False, tie_tol=0.0, fp64_final=False):
    """Damped IsoRank of every pair (cfsim_score_damped): run once, synchronise,
    return (results, matches, S list).  prior: None (uniform) or one n_B x n_A
    array per pair."""
    b = Batch(ctx, gs, pair_a, pair_b, dtype, max_iter, tol, "none", want_match, want_S, path="damped",
              tie_tol=tie_tol, fp64_final=fp64_final, alpha=alpha, prior=prior)
    b.run()
    torch.cuda.synchronize()
    return b.results(), (b.matches() if want_match else None), (b.S_list() if want_S else None)


def assign(ctx, S_list, dtype="f64", stream=None):
    """Optimal-assignment matching (cfsim_assign) of host matrices: returns
    (list of row -> column arrays, scores)."""
    mats = [np.asarray(x) for x in S_list]
    npdt = np.float64 if dtype == "f64" else np.float32
    flat = np.concatenate([m.astype(npdt).ravel() for m in mats]) if mats else np.zeros(1, npdt)
    off = np.concatenate([[0], np.cumsum([m.size for m in mats])]).astype(np.int64)
    nr = np.array([m.shape[0] for m in mats], np.int32)
    nc = np.array([m.shape[1] for m in mats], np.int32)
    moff = np.concatenate([[0], np.cumsum(nr)]).astype(np.int64)
    dev = torch.device("cuda", ctx.device)
    t = lambda a: torch.as_tensor(a).to(dev)
    dS, dSo, dnr, dnc, dmo = t(flat), t(off[:-1]), t(nr), t(nc), t(moff[:-1])
    match = torch.empty(max(int(moff[-1]), 1), dtype=torch.int32, device=dev)
    scores = torch.empty(max(len(mats), 1), dtype=torch.float64, device=dev)
    max_dim = int(max([max(m.shape) for m in mats], default=1))
    _check(lib().cfsim_assign(ctx.handle, F64 if dtype == "f64" else F32, _ptr(dS), _ptr(dSo), _ptr(dnr), _ptr(dnc),
                              len(mats), max_dim, _ptr(match), _ptr(dmo), _ptr(scores), _stream(stream)))
    torch.cuda.synchronize()
    m = match.cpu().numpy()
    return [m[o:o + r] for o, r in zip(moff[:-1], nr)], scores[: len(mats)].cpu().numpy()


def ward(ctx, X, stream=None) -> torch.Tensor:
    """Ward's clustering of the rows of X (cfsim_ward): the (n - 1) x 4 FP64
    linkage matrix on the device.  X: host array or FP64 device tensor."""
    dev = torch.device("cuda", ctx.device)
    Xd = X.to(device=dev, dtype=torch.float64).contiguous() if isinstance(X, torch.Tensor) else \
        torch.as_tensor(np.ascontiguousarray(X, np.float64)).to(dev)
    n, f = int(Xd.shape[0]), int(Xd.shape[1])
    Z = torch.empty((max(n - 1, 1), 4), dtype=torch.float64, device=dev)
    ws_bytes = lib().cfsim_ward_workspace_size(n)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)
    _check(lib().cfsim_ward(ctx.handle, _ptr(Xd), n, f, _ptr(Z), _ptr(ws), ws_bytes, _stream(stream)))
    return Z[: max(n - 1, 0)]
