#!/usr/bin/env python3
"""Benchmark: CFG-pair similarities per second on one MI355X, batched vs plain.

Workload: 256 synthetic CFGs (node counts uniform in [8, 128], loop trip
counts log-uniform in [1, 1e4]), all 32,640 unordered pairs, FP32 with FP64
reductions, tol 1e-12, at most 200 iterations.  A step is one batched pass
over every pair (one replay of the cached HIP graph: device-side plan plus
the persistent size-bucketed pair kernels), scores and matchings written to
device memory; inputs are resident in HBM before the timed region.

Prints one JSON line.  Besides the contract fields it reports the plain path
(one cfsim_score launch per pair, same dtype), the error of every FP32 pair
against the FP64 GPU path (itself parity-tested against the CPU oracle), an
oracle check on a seeded sample, the roofline of the batched pass, and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12        # MI355X FP32 vector FLOP/s (published)
LDS_PEAK = 256 * 128 * 2.4e9       # 256 CUs x 128 B/clk x 2.4 GHz


def _cpu_worker(args):
    """Oracle on a chunk of pairs (runs in a child process, BLAS single-threaded)."""
    pairs, seed = args
    import oracle
    from cfgsynth import config_graphs
    w = config_graphs(1)
    g = w["graphs"]
    t0 = time.perf_counter()
    for p in pairs:
        ga, gb = g[w["pair_a"][p]], g[w["pair_b"][p]]
        A = oracle.transition_matrix(ga.n, ga.src, ga.dst, ga.count)
        B = oracle.transition_matrix(gb.n, gb.src, gb.dst, gb.count)
        oracle.score_pair(A, B, 200, 1e-12)
    return time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_pairs_total: int, sample: int, seed: int = 7, gpu_S=None):
    """The oracle as it stands, on a bounded seeded sample, across host cores
    (at most 16 processes: the host share of one GPU).  gpu_S, if given, maps
    a pair index to its (FP32, FP64) GPU S: the oracle S of 16 seeded pairs is
    then compared with them after the timed part."""
    import multiprocessing as mp
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    rng = np.random.default_rng(seed)
    idx = rng.choice(n_pairs_total, size=sample, replace=False)
    chunks = [(idx[i::cores].tolist(), seed) for i in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        busy = pool.map(_cpu_worker, chunks)
    wall = time.perf_counter() - t0
    out = dict(value=sample / wall, unit="pairs/s", cores=cores, kind="oracle", cpu_model=cpu_model(),
               sample=f"{sample} seeded pairs of the 32,640 (FP64 NumPy oracle, tol 1e-12, <=200 iterations), "
                      f"{cores} processes, {sum(busy):.1f} s of CPU work, {wall:.1f} s wall")
    if gpu_S is not None:
        import oracle
        from cfgsynth import config_graphs
        w = config_graphs(1)
        g = w["graphs"]
        orng = np.random.default_rng(5)
        e32, e64 = [], []
        for p in orng.choice(n_pairs_total, size=16, replace=False):
            ga, gb = g[w["pair_a"][p]], g[w["pair_b"][p]]
            ref = oracle.score_pair(oracle.transition_matrix(ga.n, ga.src, ga.dst, ga.count),
                                    oracle.transition_matrix(gb.n, gb.src, gb.dst, gb.count), 200, 1e-12)
            S32, S64 = gpu_S(int(p))
            scale = np.max(np.abs(ref.S))
            e32.append(float(np.max(np.abs(S32.astype(np.float64) - ref.S)) / scale))
            e64.append(float(np.max(np.abs(S64 - ref.S)) / scale))
        out["oracle_check"] = dict(pairs=16, max_elementwise_err_fp32=max(e32), max_elementwise_err_fp64=max(e64),
                                   gate_pass=bool(max(e32) <= 1e-5 and max(e64) <= 1e-10))
    return out


def kernel_sources_digest() -> str:
    """SHA-256 over the sources the batched pair kernels are built from
    (detects kernels changed since their counters were taken)."""
    import hashlib
    d = os.path.join(ROOT, "paper_1707_02423_amd", "csrc")
    h = hashlib.sha256()
    for name in ("cfsim_internal.h", "pair_device.h", "pair.hip"):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def traffic_of(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if there is none or
    the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_workload1.txt")
    if not os.path.exists(path):
        return None
    digest, found = None, None
    with open(path) as f:
        for ln in f:
            parts = ln.split()
            if len(parts) == 2 and parts[0] == "source_sha256":
                digest = parts[1]
            elif len(parts) >= 3 and parts[0] == "traffic_bytes_per_launch" and " ".join(parts[2:]) == kernel:
                found = float(parts[1])
    return found if digest == kernel_sources_digest() else None


def plain_leg(ctx, gs, pa, pb, res, n_sub, stream):
    """One cfsim_score launch per pair on a seeded sample, same dtype."""
    import torch
    from paper_1707_02423_amd import cfsim as cfm
    rng = np.random.default_rng(11)
    sub = rng.choice(len(pa), size=min(n_sub, len(pa)), replace=False)
    L = cfm.lib()
    opt = cfm.options("f32")
    dev = gs.w.device
    maxn = int(gs.sizes().max())
    m_buf = torch.empty(maxn, dtype=torch.int32, device=dev)
    r_buf = torch.empty(len(sub) * cfm.RESULT_BYTES, dtype=torch.uint8, device=dev)
    ws_bytes = L.cfsim_score_workspace_size(ctx.handle, maxn, maxn, ctypes.byref(opt))
    ws_buf = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    gA = [gs.graph(int(pa[p])) for p in sub]
    gB = [gs.graph(int(pb[p])) for p in sub]
    sh = stream.cuda_stream

    def plain_pass():
        for k in range(len(sub)):
            rc = L.cfsim_score(ctx.handle, ctypes.byref(gA[k]), ctypes.byref(gB[k]), ctypes.byref(opt), None,
                               m_buf.data_ptr(), r_buf.data_ptr() + cfm.RESULT_BYTES * k, ws_buf.data_ptr(), ws_bytes, sh)
            if rc != 0:
                raise RuntimeError(L.cfsim_last_error().decode())
    plain_pass()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    plain_pass()
    ev1.record(stream)
    torch.cuda.synchronize()
    plain_ms = ev0.elapsed_time(ev1)
    plain_res = r_buf.cpu().numpy().view(cfm.RESULT_DTYPE)
    return dict(plain_value=len(sub) / (plain_ms * 1e-3), plain_pairs_timed=int(len(sub)),
                plain_vs_batched_max_score_diff=float(np.max(np.abs(plain_res["score"] - res["score"][sub]))))


def _time_ms(fn, reps, stream):
    """Average milliseconds of fn() over reps calls (HIP events on `stream`)."""
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def seg_errors(Sa, Sb, counts):
    """Per-pair errors of Sa (FP32, flat) against Sb (FP64, flat; pair p owns
    counts[p] consecutive entries): relative Frobenius error, max |dS| over
    max |Sb| (element-wise), and the largest |dS| / Sb over the entries FP32
    holds with full precision (Sb >= 1e-30)."""
    import torch
    dev = Sb.device
    n = len(counts)
    seg = torch.repeat_interleave(torch.arange(n, device=dev), torch.as_tensor(np.asarray(counts, np.int64), device=dev))
    m = seg.numel()
    d = Sa[:m].double() - Sb[:m]
    B = Sb[:m]
    z = lambda: torch.zeros(n, dtype=torch.float64, device=dev)
    num = z().index_add_(0, seg, d * d)
    den = z().index_add_(0, seg, B * B)
    ad = d.abs()
    dmax = z().index_reduce_(0, seg, ad, "amax")
    smax = z().index_reduce_(0, seg, B.abs(), "amax")
    big = B >= 1e-30
    rel = torch.where(big, ad / torch.where(big, B, torch.ones_like(B)), torch.zeros_like(B))
    rmax = z().index_reduce_(0, seg, rel, "amax")
    frob = torch.sqrt(num / den)
    elem = dmax / smax
    return frob.cpu().numpy(), elem.cpu().numpy(), rmax.cpu().numpy()


def err_summary(frob, elem, entry):
    return dict(max_rel_err_vs_fp64=float(frob.max()), median_rel_err_vs_fp64=float(np.median(frob)),
                max_elementwise_err_vs_fp64=float(elem.max()), max_entry_rel_err_vs_fp64=float(entry.max()))


def certify(S32, m32, S64, dm, floor=1e-30):
    """The FP32 picks, in FP32 greedy order, replayed on the FP64 S: each must
    be within a relative dm of the best FP64 entry still admissible (or that
    best is below `floor`).  Returns True if every pick passes."""
    nB, nA = S64.shape
    picks = [(i, int(j)) for i, j in enumerate(m32) if j >= 0]
    picks.sort(key=lambda e: (-float(S32[e]), e[0] * nA + e[1]))
    order = np.argsort(-S64, axis=None, kind="stable")
    row_used = np.zeros(nB, bool)
    col_used = np.zeros(nA, bool)
    ptr = 0
    for i, j in picks:
        while ptr < order.size and (row_used[order[ptr] // nA] or col_used[order[ptr] % nA]):
            ptr += 1
        best = float(S64.flat[order[ptr]])
        if not (S64[i, j] >= best * (1.0 - dm) or best < floor):
            return False
        row_used[i] = True
        col_used[j] = True
    return True


def plain_pair_leg(ctx, stream, reps=200):
    """The plain method on the 12 x 16 pair (FP64, and FP32 for reference):
    one cfsim_score launch per pair, back to back; microseconds per pair and
    nanoseconds per update."""
    import torch
    import paper_1707_02423_amd as cf
    from paper_1707_02423_amd import cfsim as cfm
    from cfgsynth import config_graphs
    w = config_graphs(0)
    gs = cf.pack(ctx, w["graphs"])
    L = cfm.lib()
    A, B = gs.graph(0), gs.graph(1)
    out = dict(workload="one pair of synthetic CFGs, 12 and 16 nodes, branch counts U[1,1000], tol 1e-12, "
                        "<=200 updates, one cfsim_score launch per pair")
    for dt in ("f64", "f32"):
        opt = cfm.options(dt)
        res = torch.empty(cfm.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        m = torch.empty(B.n, dtype=torch.int32, device="cuda")
        wsb = L.cfsim_score_workspace_size(ctx.handle, A.n, B.n, ctypes.byref(opt))
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
        sh = stream.cuda_stream

        def one():
            rc = L.cfsim_score(ctx.handle, ctypes.byref(A), ctypes.byref(B), ctypes.byref(opt), None, m.data_ptr(),
                               res.data_ptr(), ws.data_ptr(), wsb, sh)
            if rc != 0:
                raise RuntimeError(L.cfsim_last_error().decode())
        for _ in range(10):
            one()
        torch.cuda.synchronize()
        ms = _time_ms(one, reps, stream)
        r = res.cpu().numpy().view(cfm.RESULT_DTYPE)[0]
        out[dt] = dict(us_per_pair=ms * 1e3, ns_per_update=ms * 1e6 / max(int(r["iters"]), 1),
                       iters=int(r["iters"]), status=int(r["status"]))
    return out


def workload_legs(ctx, stream, reps=3):
    """The other hot-path rows, each on its own synthetic workload: the plain
    12 x 16 pair, large pairs (tiled path), query-vs-database with top-16,
    the reverse mode, the scale-to-common-size mode of the all-pairs batch,
    the elementwise distances of Table 1, the damped IsoRank measure, the
    optimal-assignment matching and Ward's clustering.  Inputs resident in HBM; every time is the average of `reps` timed
    calls after one warm-up; every leg states its error against the FP64 GPU
    path (itself parity-tested against the CPU oracle)."""
    import torch
    import paper_1707_02423_amd as cf
    from cfgsynth import config_graphs
    out = {"plain_pair": plain_pair_leg(ctx, stream)}

    # a9: 64 pairs, 512-2048 nodes, one tiled launch sequence (HIP graph)
    w = config_graphs(2)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True, path="large")
    b.run()
    torch.cuda.synchronize()
    ms = _time_ms(b.run, reps, stream)
    r = b.results()
    nA, nB = b.nA.astype(np.float64), b.nB.astype(np.float64)
    it = r["iters"].astype(np.float64)
    # per update: read the previous iterate and write the new one (8 B per
    # entry); every other update also reads the two iterates of the change (4 B
    # per entry and update on average)
    alg_bytes = float(np.sum(it * nA * nB * (8.0 + 2.0)))
    b32 = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True, want_S=True, path="large")
    b64 = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f64", want_match=True, want_S=True, path="large")
    b32.run()
    b64.run()
    torch.cuda.synchronize()
    errs = err_summary(*seg_errors(b32.S, b64.S, b32.nA * b32.nB))
    r32 = b32.results()
    out["large_pairs"] = dict(workload="64 pairs of synthetic CFGs, n ~ U[512,2048], FP32, <=200 updates",
                              ms_per_call=ms, pairs_per_s=len(r) / (ms * 1e-3),
                              hbm_roofline=dict(bound="hbm", achieved=alg_bytes / (ms * 1e-3) / 1e9, peak=8000.0,
                                                unit="GB/s", frac=alg_bytes / (ms * 1e-3) / 8e12),
                              status_counts={int(k): int(v) for k, v in zip(*np.unique(r["status"], return_counts=True))},
                              near_tie_count=int(np.sum((r32["status"] & cf.NEAR_TIE) != 0)),
                              matchings_equal_fp32_fp64=int(sum(np.array_equal(x, y) for x, y in
                                                                zip(b32.matches(), b64.matches()))),
                              **errs)
    # the same call with block-sparse BF16 matrix-core products (FP32 sums)
    bm = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True, want_S=True, path="large",
                  mfma=True)
    bm.run()
    torch.cuda.synchronize()
    ms_m = _time_ms(bm.run, reps, stream)
    rm = bm.results()
    errs_m = err_summary(*seg_errors(bm.S, b64.S, bm.nA * bm.nB))
    # executed matrix-core work per update of a pair: stage 1 takes every
    # nonzero 32 x 32 block of A twice (A S^T, A^T S^T) per block row of S,
    # stage 2 every nonzero block of B twice per block column; two 32x32x16
    # MFMAs (32,768 flops each) per block product
    def nblocks(g):
        return len(set(zip((np.asarray(g.src) // 32).tolist(), (np.asarray(g.dst) // 32).tolist())))
    gr = w["graphs"]
    ex = 0.0
    for p in range(len(w["pair_a"])):
        ga, gb = gr[w["pair_a"][p]], gr[w["pair_b"][p]]
        nRb, nCb = (gb.n + 31) // 32, (ga.n + 31) // 32
        ex += float(rm["iters"][p]) * (nRb * 2 * nblocks(ga) + nCb * 2 * nblocks(gb)) * 2 * 32768.0
    out["large_pairs"]["mfma_bf16"] = dict(
        ms_per_call=ms_m, pairs_per_s=len(rm) / (ms_m * 1e-3), speedup_over_fp32=ms / ms_m,
        mfma_roofline=dict(bound="mfma", executed_tflops=ex / 1e12, achieved=ex / (ms_m * 1e-3) / 1e12,
                           peak=2500.0, unit="TFLOP/s", frac=ex / (ms_m * 1e-3) / 2.5e15),
        status_counts={int(k): int(v) for k, v in zip(*np.unique(rm["status"], return_counts=True))},
        matchings_equal_fp64=int(sum(np.array_equal(x, y) for x, y in zip(bm.matches(), b64.matches()))),
        **errs_m)
    del b, b32, b64, bm, gs

    # a8 + a11: a 200-node query against 65,536 power-law graphs, then top-16
    w = config_graphs(4)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=False)
    b.run()
    b.topk(16)
    torch.cuda.synchronize()
    ms = _time_ms(b.run, reps, stream)
    ms_topk = _time_ms(lambda: b.topk(16), reps, stream)
    i32, _ = b.topk(16)
    b32 = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True, want_S=True)
    b64 = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f64", want_match=True, want_S=True)
    b32.run()
    b64.run()
    i64, _ = b64.topk(16)
    torch.cuda.synchronize()
    errs = err_summary(*seg_errors(b32.S, b64.S, b32.nA * b32.nB))
    out["query_db"] = dict(workload="200-node query vs 65,536 CFGs (p(n) ~ n^-2 on [4,512]), FP32, top-16",
                           ms_per_call=ms, pairs_per_s=len(w["pair_a"]) / (ms * 1e-3), topk_ms=ms_topk,
                           top16_equal_fp64=bool(torch.equal(i32, i64)),
                           near_tie_count=int(np.sum((b32.results()["status"] & cf.NEAR_TIE) != 0)),
                           matchings_equal_fp32_fp64=int(sum(np.array_equal(x, y) for x, y in
                                                             zip(b32.matches(), b64.matches()))),
                           **errs)
    del b, b32, b64, gs

    # a10: 1,024 pairs n ~ U[16,256], forward then reverse mode (checkpoints every 8)
    w = config_graphs(3)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True, checkpoint_every=8)
    b.run()
    gsc = torch.ones(len(w["pair_a"]), dtype=torch.float64, device=gs.w.device)
    gw = torch.zeros_like(gs.w)
    st = cf.backward(b, gsc, gw, checkpoint_every=8)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(st)) == 0, "the reverse mode skipped pairs"
    ms_f = _time_ms(b.run, reps, stream)
    ms_b = _time_ms(lambda: cf.backward(b, gsc, gw, checkpoint_every=8), reps, stream)
    g32 = torch.zeros_like(gs.w)
    cf.backward(b, gsc, g32, checkpoint_every=8)
    b64 = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f64", want_match=True, checkpoint_every=8)
    b64.run()
    g64 = torch.zeros_like(gs.w)
    st64 = cf.backward(b64, gsc, g64, checkpoint_every=8)
    torch.cuda.synchronize()
    same = np.array([np.array_equal(x, y) for x, y in zip(b.matches(), b64.matches())])
    # pairs with the same matching have the same derivative up to rounding
    eidx = np.concatenate([np.arange(gs.edge_off[g], gs.edge_off[g + 1]) for p in np.flatnonzero(same)
                           for g in (int(w["pair_a"][p]), int(w["pair_b"][p]))])
    e = torch.as_tensor(eidx, device=gs.w.device)
    gerr = float(torch.linalg.norm(g32[e] - g64[e]) / torch.linalg.norm(g64[e]))
    out["backward"] = dict(workload="1,024 pairs n ~ U[16,256], FP32, gradient w.r.t. every edge weight, "
                                    "forward with checkpoints every 8 updates",
                           forward_ms=ms_f, backward_ms=ms_b,
                           pairs_per_s_fwd_bwd=len(w["pair_a"]) / ((ms_f + ms_b) * 1e-3),
                           backward_over_forward=ms_b / ms_f, pairs_skipped=int(torch.count_nonzero(st)),
                           pairs_same_matching_fp32_fp64=int(same.sum()),
                           grad_rel_err_vs_fp64=gerr, fp64_pairs_skipped=int(torch.count_nonzero(st64)))
    del b, b64, gs

    # a2: the all-pairs batch with the bilinear scale to a common size
    w = config_graphs(1)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", resize="bilinear", want_match=True, want_S=True)
    b.run()
    torch.cuda.synchronize()
    ms = _time_ms(b.run, max(1, reps - 1), stream)
    b64 = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f64", resize="bilinear", want_match=True, want_S=True)
    b64.run()
    torch.cuda.synchronize()
    errs = err_summary(*seg_errors(b.S, b64.S, b.nA * b.nB))
    out["resize"] = dict(workload="all 32,640 pairs of the 256-CFG batch, bilinear scale to a common size, FP32",
                         ms_per_call=ms, pairs_per_s=len(w["pair_a"]) / (ms * 1e-3),
                         near_tie_count=int(np.sum((b.results()["status"] & cf.NEAR_TIE) != 0)),
                         matchings_equal_fp32_fp64=int(sum(np.array_equal(x, y) for x, y in
                                                           zip(b.matches(), b64.matches()))),
                         **errs)
    del b, b64, gs

    # f1: Table 1's five elementwise distances (Minkowski p = 3) of every pair
    # of the 256-CFG batch and of the 64 large pairs, FP64.  Work per entry of
    # the M x M common-size matrices: the interpolated entry (9 flops) and
    # the six sums (13 flops).
    dist = {}
    for key, idx, label in (("all_pairs", 1, "all 32,640 pairs of the 256-CFG batch, n ~ U[8,128]"),
                            ("large_pairs", 2, "64 pairs of synthetic CFGs, n ~ U[512,2048]")):
        w = config_graphs(idx)
        gs = cf.pack(ctx, w["graphs"])
        dev = gs.w.device
        pa = torch.as_tensor(w["pair_a"], device=dev)
        pb = torch.as_tensor(w["pair_b"], device=dev)
        d = cf.distances(ctx, gs, pa, pb, stream=stream)
        torch.cuda.synchronize()
        ms = _time_ms(lambda: cf.distances(ctx, gs, pa, pb, stream=stream), reps, stream)
        sizes = np.diff(gs.node_off).astype(np.float64)
        M = np.maximum(sizes[w["pair_a"]], sizes[w["pair_b"]])
        entries = float(np.sum(M * M))
        tflops = 22.0 * entries / (ms * 1e-3) / 1e12
        dist[key] = dict(workload=label + ", five distances on the common-size matrices, FP64",
                         ms_per_call=ms, pairs_per_s=len(w["pair_a"]) / (ms * 1e-3),
                         entries_per_s=entries / (ms * 1e-3),
                         alu_roofline=dict(bound="alu", achieved=tflops, peak=78.6, unit="TFLOP/s",
                                           frac=tflops / 78.6),
                         all_finite=bool(torch.isfinite(d).all()))
        del gs, d
    out["distances"] = dist

    # f2: damped IsoRank (alpha = 0.85, uniform prior) of every pair of the
    # 256-CFG batch, FP32 against the FP64 GPU path.  Work per update: the
    # gather over Z = x / d (4 nnz_A nnz_B flops) and per entry the division
    # by d, the damped update, the 1-norm change and the squared norm (7 flops).
    w = config_graphs(1)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True, want_S=True, path="damped",
                 alpha=0.85)
    b.run()
    torch.cuda.synchronize()
    ms = _time_ms(b.run, reps, stream)
    b64 = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f64", want_match=True, want_S=True, path="damped",
                   alpha=0.85)
    b64.run()
    torch.cuda.synchronize()
    r32, r64 = b.results(), b64.results()
    errs = err_summary(*seg_errors(b.S, b64.S, b.nA * b.nB))
    nnz = np.diff(gs.edge_off).astype(np.float64)
    ea, eb = nnz[w["pair_a"]], nnz[w["pair_b"]]
    flops = float(np.sum(r32["iters"].astype(np.float64) * (4.0 * ea * eb + 7.0 * b.nA * b.nB)))
    tf = flops / (ms * 1e-3) / 1e12
    out["damped"] = dict(workload="all 32,640 pairs of the 256-CFG batch, damped IsoRank alpha = 0.85, uniform "
                                  "prior, FP32, tol 1e-12 on the 1-norm step, <=200 updates",
                         ms_per_call=ms, pairs_per_s=len(w["pair_a"]) / (ms * 1e-3),
                         alu_roofline=dict(bound="alu", achieved=tf, peak=157.3, unit="TFLOP/s", frac=tf / 157.3),
                         iters_fp64_median=float(np.median(r64["iters"])),
                         near_tie_count=int(np.sum((r32["status"] & cf.NEAR_TIE) != 0)),
                         matchings_equal_fp32_fp64=int(sum(np.array_equal(x, y) for x, y in
                                                           zip(b.matches(), b64.matches()))),
                         **errs)
    del b, b64, gs

    # f3: optimal-assignment matching of every pair's FP32 S of the 256-CFG
    # batch (the batched path's S_out), against the greedy matching's score
    w = config_graphs(1)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True, want_S=True)
    b.run()
    b.assign()
    torch.cuda.synchronize()
    ms = _time_ms(b.assign, reps, stream)
    _, sc = b.assign()
    torch.cuda.synchronize()
    sc = sc.cpu().numpy()
    greedy = b.results()["score"]
    gain = sc / greedy - 1.0
    out["assignment"] = dict(workload="optimal assignment (Hungarian, FP64 potentials) of the FP32 S of all 32,640 "
                                      "pairs of the 256-CFG batch, one wave per matrix",
                             ms_per_call=ms, pairs_per_s=len(sc) / (ms * 1e-3), all_finite=bool(np.isfinite(sc).all()),
                             pairs_above_greedy=int(np.sum(gain > 1e-6)), max_gain_over_greedy=float(gain.max()),
                             mean_gain_over_greedy=float(gain.mean()), min_gain_over_greedy=float(gain.min()))
    del b, gs

    # f4: Ward's clustering (squared Euclidean distances, Lance-Williams
    # merges) of the 256 graphs, each described by its row of the all-pairs
    # FP32 score matrix (self pairs on the diagonal); and of 4,096 seeded
    # points with 16 features (the largest size one workgroup's merge state
    # holds)
    w = config_graphs(1)
    G = len(w["graphs"])
    gs = cf.pack(ctx, w["graphs"])
    ia, ib = np.triu_indices(G)
    b = cf.Batch(ctx, gs, ia.astype(np.int32), ib.astype(np.int32), dtype="f32", want_match=False)
    b.run()
    torch.cuda.synchronize()
    sc = b.results()["score"]
    M = np.zeros((G, G))
    M[ia, ib] = sc
    M[ib, ia] = sc
    Md = torch.as_tensor(M).to(gs.w.device)
    cf.ward(ctx, Md, stream=stream)
    torch.cuda.synchronize()
    ms = _time_ms(lambda: cf.ward(ctx, Md, stream=stream), reps, stream)
    Xr = torch.as_tensor(np.random.default_rng(170702423).random((4096, 16))).to(gs.w.device)
    cf.ward(ctx, Xr, stream=stream)
    torch.cuda.synchronize()
    ms_big = _time_ms(lambda: cf.ward(ctx, Xr, stream=stream), 1, stream)
    out["ward"] = dict(workload="Ward clustering of the 256 graphs by their rows of the all-pairs FP32 score matrix "
                                "(256 features); and of 4,096 seeded points with 16 features",
                       ms_per_call=ms, merges_per_s=(G - 1) / (ms * 1e-3), ms_4096_points=ms_big)
    del b, gs
    return out


def profile_only(spec: str):
    """Launch drivers for profilers; inputs as in the bench, results unchecked:
      pair:NA:NB:DTYPE:MAX_ITER:REPS  the plain path on one seeded pair
                                      (tol 0: every launch runs MAX_ITER updates)
      workload:NAME:REPS              NAME = batch, large, largemfma, resize,
                                      query, backward, fp64final, damped or
                                      assign (FP32; assign times cfsim_assign
                                      on the batch's S), or
                                      distances / distlarge (the elementwise
                                      distances of the batch / the large pairs,
                                      FP64); REPS calls after one warm-up"""
    import torch
    from paper_1707_02423_amd import cfsim as cfm
    from cfgsynth import Grammar, config_graphs, make_cfg
    ctx = cfm.Context(0)
    f = spec.split(":")
    if f[0] == "pair" and len(f) == 6:
        na, nb, dt, K, reps = int(f[1]), int(f[2]), f[3], int(f[4]), int(f[5])
        rng = np.random.default_rng(1)
        graphs = [make_cfg(na, Grammar(counts="trip"), rng), make_cfg(nb, Grammar(counts="trip"), rng)]
        gs = cfm.pack(ctx, graphs)
        for _ in range(reps):
            cfm.score(ctx, gs, 0, 1, dtype=dt, max_iter=K, tol=0.0, want_S=False, sync=False)
    elif f[0] == "workload" and len(f) == 3:
        name, reps = f[1], int(f[2])
        idx = {"batch": 1, "resize": 1, "fp64final": 1, "large": 2, "largemfma": 2, "backward": 3,
               "query": 4, "distances": 1, "distlarge": 2, "damped": 1, "assign": 1}.get(name)
        if idx is None:
            raise SystemExit(f"unknown workload {name!r}")
        if name in ("distances", "distlarge"):
            w = config_graphs(idx)
            gs = cfm.pack(ctx, w["graphs"])
            pa = torch.as_tensor(w["pair_a"], device=gs.w.device)
            pb = torch.as_tensor(w["pair_b"], device=gs.w.device)
            for _ in range(reps + 1):
                cfm.distances(ctx, gs, pa, pb)
            torch.cuda.synchronize()
            print("done", spec, flush=True)
            return
        w = config_graphs(idx)
        kw = dict(path="large") if name in ("large", "largemfma") else {}
        kw.update(dict(mfma=True) if name == "largemfma" else {})
        kw.update(dict(resize="bilinear") if name == "resize" else {})
        kw.update(dict(fp64_final=True) if name == "fp64final" else {})
        kw.update(dict(path="damped", alpha=0.85) if name == "damped" else {})
        kw.update(dict(want_S=True) if name == "assign" else {})
        gs = cfm.pack(ctx, w["graphs"])
        b = cfm.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True, **kw)
        gsc = torch.ones(b.n_pairs, dtype=torch.float64, device=gs.w.device)
        gw = torch.zeros_like(gs.w)
        if name == "assign":
            b.run()
        for _ in range(reps + 1):
            if name == "assign":
                b.assign()
                continue
            b.run()
            if name == "backward":
                cfm.backward(b, gsc, gw)
    else:
        raise SystemExit(profile_only.__doc__)
    torch.cuda.synchronize()
    print("done", spec, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-pairs", type=int, default=1024)
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=3, help="timed eager passes for per-kernel durations")
    ap.add_argument("--no-legs", action="store_true", help="skip the other workloads (large pairs, query, ...)")
    ap.add_argument("--no-tune", action="store_true", help="time the default plan (no autotuning)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device copy of this size first (profiler byte-counter calibration)")
    ap.add_argument("--only", default="", help="profiling driver instead of the bench (see profile_only)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); pairs would shard across GPUs "
              "by cost with one persistent launch per GPU, which this build does not run.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1707_02423_amd as cf
    from cfgsynth import config_graphs

    if args.copy_calibration_mib > 0:
        src = torch.ones(args.copy_calibration_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        profile_only(args.only)
        return

    w = config_graphs(1)
    graphs, pa, pb = w["graphs"], w["pair_a"], w["pair_b"]
    n_pairs = len(pa)
    ctx = cf.Context(0)
    gs = cf.pack(ctx, graphs)
    torch.cuda.synchronize()

    # ---------------------------------------------------------------- plan autotuning (untimed)
    tune_rec = None
    if not args.no_tune:
        from paper_1707_02423_amd import tune
        tune_rec = tune.autotune(ctx, gs, pa, pb, "f32", reps=3)
        tune.save(tune_rec)

    # ---------------------------------------------------------------- batched
    batch = cf.Batch(ctx, gs, pa, pb, dtype="f32", want_match=True, want_S=False)
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        batch.run()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    value = n_pairs / (ms * 1e-3)
    res = batch.results()
    iters = res["iters"].astype(np.float64)
    sizes = gs.sizes()
    nnz = np.diff(gs.edge_off)
    nA, nB = sizes[pa].astype(np.float64), sizes[pb].astype(np.float64)
    mA, mB = nnz[pa].astype(np.float64), nnz[pb].astype(np.float64)
    pair_flops = iters * (4.0 * mA * mB + 3.0 * nA * nB)
    flops = float(np.sum(pair_flops))
    lds_bytes = float(np.sum(iters * (2.0 * mA * mB + nA * nB) * 4.0))
    achieved = flops / (ms * 1e-3)

    # ---------------------------------------------------------------- dominant kernel
    # Same launches without the graph, with an event pair on each bucket's
    # stream around its kernel; the dominant kernel is the longest bucket.
    bucket = batch.buckets()
    ctx.set_timing(True)
    kms = np.zeros(cf.NUM_BUCKETS)
    for _ in range(args.kernel_reps):
        batch.run()
        kms += ctx.batch_timings()
    ctx.set_timing(False)
    kms /= args.kernel_reps
    dom = int(np.argmax(kms[:cf.NUM_BUCKETS - 1]))
    dom_flops = float(np.sum(pair_flops[bucket == dom]))
    dom_achieved = dom_flops / (kms[dom] * 1e-3)
    kernels = {cf.bucket_kernel(v, "f32"): dict(avg_ms=float(kms[v]), pairs=int(np.sum(bucket == v)),
                                                flops=float(np.sum(pair_flops[bucket == v])))
               for v in range(cf.NUM_BUCKETS - 1) if np.any(bucket == v)}

    # ---------------------------------------------------------------- plain
    plain = {}
    if args.plain_pairs > 0:
        plain = plain_leg(ctx, gs, pa, pb, res, args.plain_pairs, stream)
        plain["batched_over_plain"] = value / plain["plain_value"]
    dev = gs.w.device

    # ---------------------------------------------------------------- verification
    ver, gpu_S = {}, None
    if not args.no_verify:
        b32 = cf.Batch(ctx, gs, pa, pb, dtype="f32", want_match=True, want_S=True)
        b64 = cf.Batch(ctx, gs, pa, pb, dtype="f64", want_match=True, want_S=True)
        b32.run()
        b64.run()
        torch.cuda.synchronize()
        r32, r64 = b32.results(), b64.results()
        assert np.array_equal(r32["score"], res["score"]), "verification run differs from the timed run"
        frob, elem, entry = seg_errors(b32.S, b64.S, b32.nA * b32.nB)
        m32, m64 = b32.matches(), b64.matches()
        same = np.array([np.array_equal(x, y) for x, y in zip(m32, m64)])
        near = (r32["status"] & cf.NEAR_TIE) != 0
        # every FP32 matching that differs from FP64's: flagged, and certified
        # on the CPU against the FP64 S (delta_m = twice the pair's largest
        # per-entry relative error)
        S32h, S64h = b32.S.cpu().numpy(), b64.S.cpu().numpy()

        S_off_h, nA_h, nB_h = np.array(b32.S_off_h), np.array(b32.nA), np.array(b32.nB)

        def pair_S(p):
            o, a, b_ = int(S_off_h[p]), int(nA_h[p]), int(nB_h[p])
            return S32h[o:o + a * b_].reshape(b_, a), S64h[o:o + a * b_].reshape(b_, a)
        diff = np.flatnonzero(~same)
        certified = 0
        for p in diff:
            S32p, S64p = pair_S(p)
            certified += certify(S32p, m32[p], S64p, max(2.0 * float(entry[p]), 1e-12))
        gpu_S = pair_S
        # the FP64 pass over the near-tie pairs (CFSIM_FLAG_FP64_FINAL)
        bf = cf.Batch(ctx, gs, pa, pb, dtype="f32", want_match=True, fp64_final=True)
        bf.run()
        torch.cuda.synchronize()
        ms_f = _time_ms(bf.run, 3, stream)
        rf = bf.results()
        same_f = int(sum(np.array_equal(x, y) for x, y in zip(bf.matches(), m64)))
        hist = {int(k): int(v) for k, v in zip(*np.unique(r32["iters"], return_counts=True))}
        ver = dict(err_summary(frob, elem, entry),
                   gate_1e5_pass=bool(frob.max() <= 1e-5 and elem.max() <= 1e-5),
                   matchings_equal_fp32_fp64=int(same.sum()),
                   near_tie_count=int(near.sum()), near_tie_tol=2e-5,
                   matching_differences=dict(pairs=int(diff.size), flagged_near_tie=int(near[diff].sum()),
                                             certified=int(certified)),
                   fp64_final=dict(ms_per_call=ms_f, pairs_per_s=n_pairs / (ms_f * 1e-3),
                                   pairs_recomputed=int(np.sum((rf["status"] & cf.FP64_FINAL) != 0)),
                                   matchings_equal_fp64=same_f),
                   iterations_histogram=hist,
                   status_counts={int(k): int(v) for k, v in zip(*np.unique(r32["status"], return_counts=True))})
        del b32, b64, bf

    line = {
        "metric": "CFG-pair similarities/sec, batched vs plain on 1 GPU, at <=1e-5 rel err vs FP64",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "wall_s_timed": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "all-pairs batch: 256 synthetic CFGs, n ~ U[8,128], loop trips log-uniform "
                               "[1,1e4], 32,640 pairs, FP32 with FP64 reductions, tol 1e-12, max 200 iterations, "
                               "one HIP-graph replay of the persistent bucketed launch (autotuned plan)",
                   "pairs": n_pairs, "graphs": len(graphs), "seed": int(w["seed"])},
        "roofline": {"bound": "alu", "achieved": dom_achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": dom_achieved / FP32_VECTOR_PEAK,
                     "traffic": traffic_of(cf.bucket_kernel(dom, "f32")),
                     "kernel": cf.bucket_kernel(dom, "f32"), "avg_launch_ms": float(kms[dom]),
                     "flops_per_launch": dom_flops},
        "step_roofline": {"achieved": achieved / 1e12, "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK},
        "kernels": kernels,
        "lds_roofline": {"achieved": lds_bytes / (ms * 1e-3) / 1e12, "peak": LDS_PEAK / 1e12, "unit": "TB/s",
                         "frac": lds_bytes / (ms * 1e-3) / LDS_PEAK},
        "algorithmic_flops_per_step": flops,
    }
    if tune_rec is not None:
        line["plan_tuning"] = dict(table={str(c): v for c, v in enumerate(tune_rec["table"]) if v >= 0},
                                   default_ms_per_pass=tune_rec["base_ms"], tuned_ms_per_pass=tune_rec["tuned_ms"],
                                   classes_tried=len(tune_rec["classes"]))
    line.update(plain)
    line.update(ver)
    if not args.no_legs:
        line["workloads"] = workload_legs(ctx, stream)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n_pairs, args.cpu_sample, gpu_S=gpu_S)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
