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


def cpu_baseline(n_pairs_total: int, sample: int, seed: int = 7):
    """The oracle as it stands, on a bounded seeded sample, across host cores."""
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
    return dict(value=sample / wall, unit="pairs/s", cores=cores, kind="oracle",
                sample=f"{sample} seeded pairs of the 32,640 (FP64 NumPy oracle, tol 1e-12, <=200 iterations), "
                       f"{cores} processes, {sum(busy):.1f} s of CPU work, {wall:.1f} s wall")


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
    r_buf = torch.empty(len(sub) * 32, dtype=torch.uint8, device=dev)
    ws_bytes = L.cfsim_score_workspace_size(ctx.handle, maxn, maxn, ctypes.byref(opt))
    ws_buf = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    gA = [gs.graph(int(pa[p])) for p in sub]
    gB = [gs.graph(int(pb[p])) for p in sub]
    sh = stream.cuda_stream

    def plain_pass():
        for k in range(len(sub)):
            rc = L.cfsim_score(ctx.handle, ctypes.byref(gA[k]), ctypes.byref(gB[k]), ctypes.byref(opt), None,
                               m_buf.data_ptr(), r_buf.data_ptr() + 32 * k, ws_buf.data_ptr(), ws_bytes, sh)
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


def workload_legs(ctx, stream, reps=3):
    """The other hot-path rows, each on its own synthetic workload: large pairs
    (tiled path), query-vs-database with top-16, the reverse mode, and the
    scale-to-common-size mode of the all-pairs batch.  Inputs resident in HBM;
    every figure is the average of `reps` timed calls after one warm-up."""
    import torch
    import paper_1707_02423_amd as cf
    from cfgsynth import config_graphs
    out = {}

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
    # per update: read the previous iterate and write the new one (8 B per entry),
    # plus the two iterates of the even-step change every other update
    alg_bytes = float(np.sum(it * nA * nB * (8.0 + 4.0)))
    out["large_pairs"] = dict(workload="64 pairs of synthetic CFGs, n ~ U[512,2048], FP32, <=200 updates",
                              ms_per_call=ms, pairs_per_s=len(r) / (ms * 1e-3),
                              hbm_roofline=dict(bound="hbm", achieved=alg_bytes / (ms * 1e-3) / 1e9, peak=8000.0,
                                                unit="GB/s", frac=alg_bytes / (ms * 1e-3) / 8e12),
                              status_counts={int(k): int(v) for k, v in zip(*np.unique(r["status"], return_counts=True))})
    del b, gs

    # a8 + a11: a 200-node query against 65,536 power-law graphs, then top-16
    w = config_graphs(4)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=False)
    b.run()
    b.topk(16)
    torch.cuda.synchronize()
    ms = _time_ms(b.run, reps, stream)
    ms_topk = _time_ms(lambda: b.topk(16), reps, stream)
    out["query_db"] = dict(workload="200-node query vs 65,536 CFGs (p(n) ~ n^-2 on [4,512]), FP32, top-16",
                           ms_per_call=ms, pairs_per_s=len(w["pair_a"]) / (ms * 1e-3), topk_ms=ms_topk)
    del b, gs

    # a10: 1,024 pairs n ~ U[16,256], forward then reverse mode (checkpoints every 8)
    w = config_graphs(3)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True)
    b.run()
    gsc = torch.ones(len(w["pair_a"]), dtype=torch.float64, device=gs.w.device)
    gw = torch.zeros_like(gs.w)
    cf.backward(b, gsc, gw, checkpoint_every=8)
    torch.cuda.synchronize()
    ms_f = _time_ms(b.run, reps, stream)
    ms_b = _time_ms(lambda: cf.backward(b, gsc, gw, checkpoint_every=8), reps, stream)
    out["backward"] = dict(workload="1,024 pairs n ~ U[16,256], FP32, gradient w.r.t. every edge weight",
                           forward_ms=ms_f, backward_ms=ms_b, pairs_per_s_fwd_bwd=len(w["pair_a"]) / ((ms_f + ms_b) * 1e-3))
    del b, gs

    # a2: the all-pairs batch with the bilinear scale to a common size
    w = config_graphs(1)
    gs = cf.pack(ctx, w["graphs"])
    b = cf.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", resize="bilinear", want_match=True)
    b.run()
    torch.cuda.synchronize()
    ms = _time_ms(b.run, max(1, reps - 1), stream)
    out["resize"] = dict(workload="all 32,640 pairs of the 256-CFG batch, bilinear scale to a common size, FP32",
                         ms_per_call=ms, pairs_per_s=len(w["pair_a"]) / (ms * 1e-3))
    del b, gs
    return out


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
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device copy of this size first (profiler byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); pairs would shard across GPUs "
              "by cost with one persistent launch per GPU, which this build does not run.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1707_02423_amd as cf
    from paper_1707_02423_amd import cfsim as cfm
    from cfgsynth import config_graphs

    if args.copy_calibration_mib > 0:
        src = torch.ones(args.copy_calibration_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = config_graphs(1)
    graphs, pa, pb = w["graphs"], w["pair_a"], w["pair_b"]
    n_pairs = len(pa)
    ctx = cf.Context(0)
    gs = cf.pack(ctx, graphs)
    torch.cuda.synchronize()

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
    ver = {}
    if not args.no_verify:
        b32 = cf.Batch(ctx, gs, pa, pb, dtype="f32", want_match=True, want_S=True)
        b64 = cf.Batch(ctx, gs, pa, pb, dtype="f64", want_match=True, want_S=True)
        b32.run()
        b64.run()
        torch.cuda.synchronize()
        r32, r64 = b32.results(), b64.results()
        assert np.array_equal(r32["score"], res["score"]), "verification run differs from the timed run"
        seg = torch.repeat_interleave(torch.arange(n_pairs, device=dev),
                                      torch.as_tensor((b32.nA * b32.nB).astype(np.int64), device=dev))
        d = (b32.S.double() - b64.S) ** 2
        num = torch.zeros(n_pairs, dtype=torch.float64, device=dev).index_add_(0, seg, d)
        den = torch.zeros(n_pairs, dtype=torch.float64, device=dev).index_add_(0, seg, b64.S ** 2)
        rel = torch.sqrt(num / den).cpu().numpy()
        del d, seg
        same_match = int(np.sum([np.array_equal(x, y) for x, y in zip(b32.matches(), b64.matches())]))
        # oracle on a seeded sample (FP64 GPU and FP32 GPU against the CPU oracle)
        import oracle
        orng = np.random.default_rng(5)
        osub = orng.choice(n_pairs, size=16, replace=False)
        o32, o64 = [], []
        S32, S64 = b32.S.cpu().numpy(), b64.S.cpu().numpy()
        for p in osub:
            ga, gb = graphs[pa[p]], graphs[pb[p]]
            ref = oracle.score_pair(oracle.transition_matrix(ga.n, ga.src, ga.dst, ga.count),
                                    oracle.transition_matrix(gb.n, gb.src, gb.dst, gb.count), 200, 1e-12)
            o, a, b = int(b32.S_off_h[p]), int(b32.nA[p]), int(b32.nB[p])
            nr = np.linalg.norm(ref.S)
            o32.append(np.linalg.norm(S32[o:o + a * b].reshape(b, a) - ref.S) / nr)
            o64.append(np.linalg.norm(S64[o:o + a * b].reshape(b, a) - ref.S) / nr)
        hist = {int(k): int(v) for k, v in zip(*np.unique(r32["iters"], return_counts=True))}
        ver = dict(max_rel_err_vs_fp64=float(rel.max()), median_rel_err_vs_fp64=float(np.median(rel)),
                   gate_1e5_pass=bool(rel.max() <= 1e-5 and max(o64) <= 1e-10),
                   oracle_sample_max_rel_err_fp32=float(max(o32)), oracle_sample_max_rel_err_fp64=float(max(o64)),
                   matchings_equal_fp32_fp64=same_match, iterations_histogram=hist,
                   status_counts={int(k): int(v) for k, v in zip(*np.unique(r32["status"], return_counts=True))})
        del b32, b64

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
                               "one HIP-graph replay of the persistent bucketed launch",
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
    line.update(plain)
    line.update(ver)
    if not args.no_legs:
        line["workloads"] = workload_legs(ctx, stream)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n_pairs, args.cpu_sample)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
