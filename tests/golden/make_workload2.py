"""Writes workload2_oracle.npz: FP64 oracle results of two pairs of the
large-pair workload (64 pairs of synthetic CFGs with 512-2048 nodes), the
largest and the smallest pair.  Calls only the oracle and the seeded input
generator.  Run from the repository root:  python tests/golden/make_workload2.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from cfgsynth import config_graphs  # noqa: E402

PAIRS = (62, 51)        # largest (2041 x 1946 S) and smallest (601 x 587) pair
N_SAMPLE = 16384        # seeded S positions stored per pair


def main():
    w = config_graphs(2)
    g = w["graphs"]
    out = {}
    for p in PAIRS:
        ga, gb = g[w["pair_a"][p]], g[w["pair_b"][p]]
        A = oracle.transition_matrix_sparse(ga.n, ga.src, ga.dst, ga.count)
        B = oracle.transition_matrix_sparse(gb.n, gb.src, gb.dst, gb.count)
        r = oracle.score_pair(A, B, w["max_iter"], w["tol"])
        rng = np.random.default_rng(1000 + p)
        idx = rng.choice(r.S.size, size=min(N_SAMPLE, r.S.size), replace=False).astype(np.int64)
        out[f"p{p}_shape"] = np.array(r.S.shape, np.int64)
        out[f"p{p}_meta"] = np.array([r.score, r.nu, r.delta, r.iters, r.status], np.float64)
        out[f"p{p}_match"] = np.asarray(r.match, np.int32)
        out[f"p{p}_idx"] = idx
        out[f"p{p}_val"] = r.S.reshape(-1)[idx]
        print(p, r.S.shape, r.iters, r.status, r.score)
    np.savez_compressed(os.path.join(HERE, "workload2_oracle.npz"), pairs=np.array(PAIRS, np.int32), **out)


if __name__ == "__main__":
    main()
