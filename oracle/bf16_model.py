"""CPU model of the BF16 matrix-core variant of the coupled iteration.

TEST INFRASTRUCTURE, like the rest of `oracle/`: only `tests/` and the
`cpu_baseline` leg of `bench.py` may import it; it shares no code with the
HIP library.

The variant computes the update of Table 1's "Iso" row (read as the
normalised power iteration of B (x) A + B^T (x) A^T, Section 4.2) with BF16
operands in every product, as a configuration of the large-pair workload
asks for.  This model follows the same steps in the same association, with
the operands rounded where the variant rounds them and every sum taken in
FP64 (the variant sums in FP32):

    Y_0 = S_0 = 1/sqrt(n_A n_B),  sigma_0 = 1
    T1 = bf16(bf16(Y_{k-1}) bf16(A)^T),   T2 = bf16(bf16(Y_{k-1}) bf16(A))
    Y_k = f32(f32(bf16(B) T1 + bf16(B)^T T2) * f32(sigma_{k-1}))
    nu_k = ||Y_k||,  sigma_k = 1 / nu_k,  S_k = Y_k sigma_k
    even k: delta_k = ||S_k - S_{k-2}||; stop when delta_k < tol

The weights are rounded through FP32 (FP64 -> FP32 -> BF16), as the variant
stores them.  `rounding=False` replaces every rounding by the identity, which
must reproduce the FP64 oracle (a pin of the structure).
"""
from __future__ import annotations

import numpy as np

from .cfsim_ref import DEGENERATE, CONVERGED, HIT_MAX_ITER, _has_positive


def round_bf16(x) -> np.ndarray:
    """Nearest BF16 value (ties to even) of each FP32 value of x (x is
    rounded to FP32 first), returned as float64.  Infinities and NaN pass
    through."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    special = ~np.isfinite(f)
    out[special] = f[special]
    return out


def _f32(x) -> np.ndarray:
    return np.asarray(x, np.float32).astype(np.float64)


def coupled_iteration_bf16(A, B, max_iter: int = 200, tol: float = 1e-12, rounding: bool = True):
    """The variant's iteration on dense A (n_A x n_A) and B (n_B x n_B).

    Returns (S, nu, delta, iters, status) like `coupled_iteration`."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    nA, nB = A.shape[0], B.shape[0]
    rb = round_bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    r32 = _f32 if rounding else (lambda v: np.asarray(v, np.float64))
    c0 = 1.0 / np.sqrt(nA * nB)
    S0 = np.full((nB, nA), float(r32(c0)))
    if not (_has_positive(A) and _has_positive(B)):
        return S0, 0.0, np.inf, 0, DEGENERATE
    Ab, Bb = rb(A), rb(B)
    Y = S0.copy()
    sigma = 1.0
    prev_even = S0
    prev_sigma_even = 1.0
    delta, nu, status, iters = np.inf, 0.0, HIT_MAX_ITER, 0
    for k in range(1, max_iter + 1):
        Sb = rb(Y)
        T1 = rb(Sb @ Ab.T)
        T2 = rb(Sb @ Ab)
        Y = r32(r32(Bb @ T1 + Bb.T @ T2) * float(r32(sigma)))
        nu = float(np.sqrt(np.sum(Y * Y)))
        sigma = 1.0 / nu
        iters = k
        if k % 2 == 0:
            cur = r32(Y * float(r32(sigma)))
            old = prev_even if k == 2 else r32(prev_even * float(r32(prev_sigma_even)))
            delta = float(np.sqrt(np.sum((cur - old) ** 2)))
            prev_even, prev_sigma_even = Y, sigma
            if delta < tol:
                status = CONVERGED
                break
    S = r32(Y * float(r32(sigma)))
    return S, nu, delta, iters, status
