"""Seeded synthetic control-flow graphs with execution counts.

This module only produces *inputs*: graph structure (basic blocks and jumps)
and integer execution counts on the edges.  It performs none of the
similarity arithmetic (no normalisation, no resize, no iteration), so both
the CPU oracle and the HIP path can consume its output.

CFG shape (paper Section 3, Background, "Kernel Control Flow Graphs"): a directed graph
with a unique START node from which every node is reachable and a unique
STOP node; nodes are basic blocks, edges are jumps.  The paper calls it
acyclic, but kernels are dominated by loops (abstract), so back-edges and
self-loops are generated.  Structure follows the structured-programming
constructs the introduction refers to: sequence, if-then, if-then-else and
loop regions.  Nodes are numbered in program (pre-)order, START is node 0,
STOP is node n-1 with no out-edges, and every node has out-degree <= 2.
"""
from __future__ import annotations

import dataclasses
import sys

import numpy as np

__all__ = ["CFG", "Grammar", "make_cfg", "config_graphs", "CONFIG_SEED_BASE",
           "power_law_sizes", "all_pairs"]

CONFIG_SEED_BASE = 170702423


@dataclasses.dataclass
class CFG:
    """One control-flow graph: n nodes and a list of weighted jumps."""
    n: int
    src: np.ndarray    # int32 [nnz], jump source (local node id)
    dst: np.ndarray    # int32 [nnz], jump target (local node id)
    count: np.ndarray  # float64 [nnz], execution count of the jump (>= 0)

    @property
    def nnz(self) -> int:
        return int(self.src.shape[0])


@dataclasses.dataclass
class Grammar:
    """Production weights and count laws of the region grammar."""
    w_seq: float = 0.40
    w_ifthen: float = 0.20
    w_ifelse: float = 0.20
    w_loop: float = 0.20
    p_selfloop: float = 0.15      # chance that a 1-node region is a self-loop
    max_loop_depth: int = 8
    # "uniform": every jump count ~ U{1..1000}.
    # "trip":    branch counts ~ U{1..1000}; a loop with trip count
    #            t = floor(10**(4u)) splits its latch as back:exit = (t-1):1.
    counts: str = "uniform"


def _draw_count(rng) -> float:
    return float(rng.integers(1, 1001))


class _Builder:
    def __init__(self, grammar: Grammar, rng):
        self.g = grammar
        self.rng = rng
        self.next_id = 0
        self.src: list[int] = []
        self.dst: list[int] = []
        self.cnt: list[float] = []

    def node(self) -> int:
        i = self.next_id
        self.next_id += 1
        return i

    def edge(self, u: int, v: int, c: float) -> None:
        self.src.append(u)
        self.dst.append(v)
        self.cnt.append(c)

    def loop_counts(self) -> tuple[float, float]:
        """(back-edge count, exit count) of a loop latch."""
        if self.g.counts == "trip":
            t = int(np.floor(10.0 ** (4.0 * self.rng.random())))
            x = _draw_count(self.rng)
            return float(t - 1) * x, x
        return _draw_count(self.rng), _draw_count(self.rng)

    def region(self, budget: int, depth: int):
        """Emit a region of exactly `budget` nodes in program order.

        Returns (entry, exit, pending) where `pending` is the count to put on
        the exit's continuation edge (decided by the loop latch law when the
        exit is a latch, else None = draw a fresh count).
        Invariant: the exit node has at most one out-edge inside the region.
        """
        g, rng = self.g, self.rng
        if budget == 1:
            b = self.node()
            if depth < g.max_loop_depth and rng.random() < g.p_selfloop:
                back, ext = self.loop_counts()
                self.edge(b, b, back)           # single-block loop body
                return b, b, ext
            return b, b, None
        choices, weights = ["seq"], [g.w_seq]
        if budget >= 3:
            choices.append("ifthen"); weights.append(g.w_ifthen)
            if depth < g.max_loop_depth:
                choices.append("loop"); weights.append(g.w_loop)
        if budget >= 4:
            choices.append("ifelse"); weights.append(g.w_ifelse)
        p = np.asarray(weights, dtype=np.float64)
        kind = choices[int(rng.choice(len(choices), p=p / p.sum()))]
        if kind == "seq":
            k = int(rng.integers(1, budget))
            e1, x1, c1 = self.region(k, depth)
            e2, x2, c2 = self.region(budget - k, depth)
            self.edge(x1, e2, c1 if c1 is not None else _draw_count(rng))
            return e1, x2, c2
        if kind == "ifthen":
            c = self.node()
            e, x, cx = self.region(budget - 2, depth)
            j = self.node()
            self.edge(c, e, _draw_count(rng))
            self.edge(c, j, _draw_count(rng))
            self.edge(x, j, cx if cx is not None else _draw_count(rng))
            return c, j, None
        if kind == "ifelse":
            c = self.node()
            k = int(rng.integers(1, budget - 2))
            e1, x1, c1 = self.region(k, depth)
            e2, x2, c2 = self.region(budget - 2 - k, depth)
            j = self.node()
            self.edge(c, e1, _draw_count(rng))
            self.edge(c, e2, _draw_count(rng))
            self.edge(x1, j, c1 if c1 is not None else _draw_count(rng))
            self.edge(x2, j, c2 if c2 is not None else _draw_count(rng))
            return c, j, None
        # loop with a latch node: body (>= 2 nodes), latch jumps back to entry
        e, x, cx = self.region(budget - 1, depth + 1)
        latch = self.node()
        self.edge(x, latch, cx if cx is not None else _draw_count(rng))
        back, ext = self.loop_counts()
        self.edge(latch, e, back)
        return e, latch, ext


def make_cfg(n: int, grammar: Grammar | None = None, rng=None, seed: int | None = None) -> CFG:
    """A CFG with exactly n >= 2 nodes: START = 0, STOP = n-1 (no out-edges)."""
    if n < 2:
        raise ValueError("a CFG needs START and STOP: n >= 2")
    grammar = grammar or Grammar()
    if rng is None:
        rng = np.random.default_rng(seed)
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 20000))
    try:
        b = _Builder(grammar, rng)
        e, x, cx = b.region(n - 1, 0)
        stop = b.node()
        b.edge(x, stop, cx if cx is not None else _draw_count(rng))
    finally:
        sys.setrecursionlimit(old)
    assert e == 0 and stop == n - 1 and b.next_id == n
    return CFG(n=n,
               src=np.asarray(b.src, dtype=np.int32),
               dst=np.asarray(b.dst, dtype=np.int32),
               count=np.asarray(b.cnt, dtype=np.float64))


def power_law_sizes(rng, count: int, lo: int, hi: int, exponent: float = 2.0) -> np.ndarray:
    """Discrete power law p(n) proportional to n**-exponent on [lo, hi]."""
    ns = np.arange(lo, hi + 1, dtype=np.float64)
    p = ns ** (-exponent)
    p /= p.sum()
    return rng.choice(np.arange(lo, hi + 1), size=count, p=p).astype(np.int64)


def all_pairs(n_graphs: int) -> tuple[np.ndarray, np.ndarray]:
    """All unordered pairs i < j, as (a = i, b = j) index arrays."""
    a, b = np.triu_indices(n_graphs, k=1)
    return a.astype(np.int32), b.astype(np.int32)


def config_graphs(index: int, scale: float = 1.0):
    """Seeded inputs of the five benchmark workloads.

    Returns a dict with "graphs" (list of CFG), "pair_a"/"pair_b" (int32
    arrays of graph indices; S is n_b x n_a), and workload parameters.
    `scale` < 1 shrinks the number of graphs/pairs (never the graph sizes)
    for quick tests.
    """
    seed = CONFIG_SEED_BASE + index
    rng = np.random.default_rng(seed)
    if index == 0:
        g = Grammar(counts="uniform")
        graphs = [make_cfg(12, g, rng), make_cfg(16, g, rng)]
        return dict(seed=seed, graphs=graphs, pair_a=np.array([0], np.int32),
                    pair_b=np.array([1], np.int32), dtype="f64", max_iter=200, tol=1e-12)
    if index == 1:
        g = Grammar(counts="trip")
        count = max(2, int(round(256 * scale)))
        sizes = rng.integers(8, 129, size=count)
        graphs = [make_cfg(int(n), g, rng) for n in sizes]
        a, b = all_pairs(count)
        return dict(seed=seed, graphs=graphs, pair_a=a, pair_b=b, dtype="f32",
                    max_iter=200, tol=1e-12)
    if index == 2:
        g = Grammar(w_seq=0.70, w_ifthen=0.08, w_ifelse=0.07, w_loop=0.15,
                    p_selfloop=0.05, max_loop_depth=4, counts="trip")
        n_pairs = max(1, int(round(64 * scale)))
        sizes = rng.integers(512, 2049, size=2 * n_pairs)
        graphs = [make_cfg(int(n), g, rng) for n in sizes]
        a = np.arange(0, 2 * n_pairs, 2, dtype=np.int32)
        return dict(seed=seed, graphs=graphs, pair_a=a, pair_b=a + 1, dtype="f32",
                    max_iter=200, tol=1e-12)
    if index == 3:
        g = Grammar(counts="trip")
        n_pairs = max(1, int(round(1024 * scale)))
        sizes = rng.integers(16, 257, size=2 * n_pairs)
        graphs = [make_cfg(int(n), g, rng) for n in sizes]
        a = np.arange(0, 2 * n_pairs, 2, dtype=np.int32)
        return dict(seed=seed, graphs=graphs, pair_a=a, pair_b=a + 1, dtype="f32",
                    max_iter=200, tol=1e-12, checkpoint_every=8)
    if index == 4:
        g = Grammar(counts="trip")
        n_db = max(1, int(round(65536 * scale)))
        query = make_cfg(200, g, rng)
        sizes = power_law_sizes(rng, n_db, 4, 512, 2.0)
        graphs = [query] + [make_cfg(int(n), g, rng) for n in sizes]
        b = np.arange(1, n_db + 1, dtype=np.int32)
        return dict(seed=seed, graphs=graphs, pair_a=np.zeros(n_db, np.int32), pair_b=b,
                    dtype="f32", max_iter=200, tol=1e-12, topk=16)
    raise ValueError(f"unknown workload index {index}")
