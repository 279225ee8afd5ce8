"""Small launch drivers for profilers (rocprofv3 kernel traces and counters).

    python3 -m paper_1707_02423_amd.probe pair NA NB DTYPE MAX_ITER REPS
        plain path (cfsim_score) on one seeded synthetic pair, REPS launches,
        tol 0 so every launch runs MAX_ITER updates
    python3 -m paper_1707_02423_amd.probe workload NAME REPS
        NAME = batch (all 32,640 pairs of the 256-CFG batch), large (64 pairs of
        512-2048 nodes on the tiled path) or resize (the batch with the bilinear
        scale to a common size); FP32, REPS calls after one warm-up

Inputs come from cfgsynth; results are not checked here (the tests do that).
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import torch

from . import cfsim as cfm


def _pair(na: int, nb: int, dtype: str, max_iter: int, reps: int):
    from cfgsynth import Grammar, make_cfg
    ctx = cfm.Context(0)
    rng = np.random.default_rng(1)
    graphs = [make_cfg(na, Grammar(counts="trip"), rng), make_cfg(nb, Grammar(counts="trip"), rng)]
    gs = cfm.pack(ctx, graphs)
    L = cfm.lib()
    A, B = gs.graph(0), gs.graph(1)
    res = torch.empty(32, dtype=torch.uint8, device="cuda")
    m = torch.empty(nb, dtype=torch.int32, device="cuda")
    opt = cfm.options(dtype, max_iter, 0.0)
    wsb = L.cfsim_score_workspace_size(ctx.handle, na, nb, ctypes.byref(opt))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    for _ in range(reps):
        rc = L.cfsim_score(ctx.handle, ctypes.byref(A), ctypes.byref(B), ctypes.byref(opt), None, m.data_ptr(),
                           res.data_ptr(), ws.data_ptr(), wsb, st)
        if rc != 0:
            raise RuntimeError(L.cfsim_last_error().decode())
    torch.cuda.synchronize()


def _workload(name: str, reps: int):
    from cfgsynth import config_graphs
    ctx = cfm.Context(0)
    if name == "large":
        w = config_graphs(2)
        kw = dict(path="large")
    elif name in ("batch", "resize"):
        w = config_graphs(1)
        kw = dict(resize="bilinear") if name == "resize" else {}
    else:
        raise SystemExit(f"unknown workload {name!r}")
    gs = cfm.pack(ctx, w["graphs"])
    b = cfm.Batch(ctx, gs, w["pair_a"], w["pair_b"], dtype="f32", want_match=True, **kw)
    for _ in range(reps + 1):
        b.run()
    torch.cuda.synchronize()


def main(argv):
    if len(argv) >= 6 and argv[0] == "pair":
        _pair(int(argv[1]), int(argv[2]), argv[3], int(argv[4]), int(argv[5]))
    elif len(argv) >= 3 and argv[0] == "workload":
        _workload(argv[1], int(argv[2]))
    else:
        raise SystemExit(__doc__)
    print("done", " ".join(argv), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
