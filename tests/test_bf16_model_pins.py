"""Pins of the CPU model of the BF16 matrix-core variant (CPU only).

* The rounding matches hand-worked BF16 values (ties to even, overflow,
  specials) and torch's FP32 -> bfloat16 conversion on random values.
* With every rounding switched off the model is the FP64 oracle's iteration
  (same S, nu, delta, update count, status): its steps and their
  association are the method's.
* With rounding, S keeps the invariants (unit norm, non-negative) and stays
  within BF16-level error of the FP64 oracle on generated CFG pairs.
* A planted mistake (the transposed term dropped) fails the structure pin.
"""
import numpy as np
import pytest

import oracle
from cfgsynth import Grammar, make_cfg


def test_round_bf16_hand_values():
    e = 2.0 ** -8
    cases = [(1.0, 1.0), (1.0 + e, 1.0), (1.0 + 3 * e, 1.0 + 4 * e), (1.0 + e + 2.0 ** -20, 1.0 + 2 * e),
             (-1.0 - 3 * e, -1.0 - 4 * e), (0.0, 0.0), (2.0 ** -130, 2.0 ** -130), (3.4e38, np.inf), (3.39e38, 3.3895313892515355e38),
             (65504.0, 65536.0), (0.1, 0.10009765625)]
    for x, want in cases:
        got = float(oracle.round_bf16(np.array([x]))[0])
        assert got == want, (x, got, want)
    sp = oracle.round_bf16(np.array([np.inf, -np.inf, np.nan]))
    assert sp[0] == np.inf and sp[1] == -np.inf and np.isnan(sp[2])


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    np.testing.assert_array_equal(oracle.round_bf16(x), ref)


def _pair(na, nb, seed):
    rng = np.random.default_rng(seed)
    ga, gb = make_cfg(na, Grammar(counts="trip"), rng), make_cfg(nb, Grammar(counts="trip"), rng)
    A = oracle.transition_matrix(ga.n, ga.src, ga.dst, ga.count)
    B = oracle.transition_matrix(gb.n, gb.src, gb.dst, gb.count)
    return A, B


@pytest.mark.parametrize("na,nb,K,tol", [(12, 16, 200, 1e-12), (40, 33, 60, 0.0), (7, 50, 200, 1e-12)])
def test_model_without_rounding_is_the_oracle(na, nb, K, tol):
    A, B = _pair(na, nb, na * 100 + nb)
    S, nu, delta, it, st = oracle.coupled_iteration_bf16(A, B, K, tol, rounding=False)
    R, rnu, rdelta, rit, rst = oracle.coupled_iteration(A, B, K, tol)
    assert it == rit and st == rst
    np.testing.assert_allclose(S, R, rtol=1e-12, atol=1e-15)
    assert abs(nu - rnu) <= 1e-12 * rnu
    if np.isfinite(rdelta):
        assert abs(delta - rdelta) <= 1e-9 * rdelta + 1e-14


def test_planted_dropped_transpose_term_fails_the_structure_pin():
    A, B = _pair(20, 24, 3)
    S = oracle.coupled_iteration_bf16(A, B, 50, 0.0, rounding=False)[0]
    # the mutant: only B S A^T (rounding off), normalised the same way
    Y = np.full(S.shape, 1.0 / np.sqrt(S.size))
    for _ in range(50):
        Y = B @ (Y @ A.T)
        nrm = np.linalg.norm(Y)
        if nrm == 0.0:
            break
        Y = Y / nrm
    R = oracle.coupled_iteration(A, B, 50, 0.0)[0]
    assert np.linalg.norm(S - R) < 1e-12
    assert np.linalg.norm(Y - R) > 1e-3


@pytest.mark.parametrize("na,nb", [(30, 45), (64, 64), (100, 70)])
def test_model_with_rounding_keeps_invariants_and_bf16_level_error(na, nb):
    A, B = _pair(na, nb, 7 * na + nb)
    S, nu, delta, it, st = oracle.coupled_iteration_bf16(A, B, 200, 1e-12)
    R = oracle.coupled_iteration(A, B, 200, 1e-12)[0]
    assert np.all(S >= 0) and abs(np.linalg.norm(S) - 1.0) < 1e-5
    err = np.linalg.norm(S - R) / np.linalg.norm(R)
    assert err < 5e-2, err
