"""Autotuner of the batched path's plan (step a8).

The batch plan runs each pair on the first LDS kernel that holds it.  A tune
table (one entry per tune class: pairs grouped by half octaves of n_A * n_B)
may send a class to a larger kernel: more threads per pair, fewer pairs per
CU.  Which is faster depends on the class and on the rest of the workload
(every bucket kernel runs to completion before the next starts), so the
tuner measures the whole batched pass: one pass of coordinate descent over
the classes present in the workload, largest first; for each class, every
kernel from the first that holds the class's pairs up to the largest is
tried, each pass timed with HIP events over `reps` graph replays after a
warm-up replay, and the fastest table is kept.  The result is cached as JSON
keyed by the GPU architecture, the arithmetic type and the class.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import cfsim as cf

NUM_LDS_KERNELS = 5


def arch_name(device: int = 0) -> str:
    """GPU architecture name without feature suffixes ("gfx950")."""
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def tune_classes(gs: cf.GraphSet, pair_a, pair_b) -> np.ndarray:
    """Tune class of every pair (the library's own classifier)."""
    sizes = gs.sizes().astype(np.int64)
    L = cf.lib()
    memo = {}
    out = np.empty(len(pair_a), np.int32)
    for p, (a, b) in enumerate(zip(np.asarray(pair_a), np.asarray(pair_b))):
        key = (int(sizes[a]), int(sizes[b]))
        if key not in memo:
            memo[key] = int(L.cfsim_tune_class(*key))
        out[p] = memo[key]
    return out


def _pass_ms(batch: cf.Batch, reps: int) -> float:
    stream = torch.cuda.current_stream()
    batch.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        batch.run()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(ctx: cf.Context, gs: cf.GraphSet, pair_a, pair_b, dtype: str = "f32", reps: int = 3,
             max_iter: int = 200, tol: float = 1e-12) -> dict:
    """Tunes the plan table of `dtype` on this workload and leaves it set in
    `ctx`.  Returns the record that `save` writes: the table, the per-class
    candidate times and the pass time before and after."""
    pair_a, pair_b = np.asarray(pair_a, np.int32), np.asarray(pair_b, np.int32)
    cls = tune_classes(gs, pair_a, pair_b)
    table = [-1] * cf.TUNE_CLASSES
    ctx.set_tune(dtype, table)
    batch = cf.Batch(ctx, gs, pair_a, pair_b, dtype=dtype, max_iter=max_iter, tol=tol, want_match=True)
    first = batch.buckets()
    base_ms = _pass_ms(batch, reps)
    best_ms = base_ms
    classes = {}
    for c in sorted(np.unique(cls).tolist(), reverse=True):
        in_c = cls == c
        lds = first[in_c][first[in_c] < NUM_LDS_KERNELS]
        if lds.size == 0:
            continue
        trial = {-1: best_ms}
        chosen = table[c]
        for v in range(int(lds.min()) + 1, NUM_LDS_KERNELS):
            table[c] = v
            ctx.set_tune(dtype, table)
            moved = batch.buckets()[in_c]
            if not np.any(moved == v):   # the kernel holds none of the class's pairs
                continue
            t = _pass_ms(batch, reps)
            trial[v] = t
            if t < best_ms:
                best_ms, chosen = t, v
        table[c] = chosen
        ctx.set_tune(dtype, table)
        classes[int(c)] = dict(pairs=int(in_c.sum()), first_kernels=sorted(set(lds.tolist())),
                               ms_per_pass={str(k): float(v) for k, v in trial.items()}, chosen=int(chosen))
    tuned_ms = _pass_ms(batch, reps)
    return dict(arch=arch_name(), dtype=dtype, table=table, classes=classes, base_ms=base_ms,
                tuned_ms=tuned_ms, pairs=int(len(pair_a)), reps=reps)


def cache_path(arch: str, dtype: str, directory: str | None = None) -> str:
    d = directory or os.environ.get("CFSIM_TUNE_DIR") or os.path.join(os.path.expanduser("~"), ".cache", "cfsim")
    return os.path.join(d, f"tune_{arch}_{dtype}.json")


def save(record: dict, directory: str | None = None) -> str:
    path = cache_path(record["arch"], record["dtype"], directory)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(record, f, indent=1, sort_keys=True)
    return path


def load(ctx: cf.Context, dtype: str = "f32", directory: str | None = None) -> dict | None:
    """Sets the cached table of this GPU's architecture and `dtype` in `ctx`
    (None, and no change, if there is none)."""
    path = cache_path(arch_name(), dtype, directory)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        record = json.load(f)
    if record.get("arch") != arch_name() or record.get("dtype") != dtype:
        return None
    ctx.set_tune(dtype, record["table"])
    return record
