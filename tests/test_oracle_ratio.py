"""Pins of the oracle's Pfaffian ratio Pf(A + U V^T - V U^T) / Pf(A).

The oracle forms the updated matrix and divides two Pfaffians.  It is pinned by
exact brute-force Pfaffians of both matrices on small integer inputs, the
closed form of a block-diagonal matrix whose one block is changed by the update,
U = V (no change), the composition of two updates, and the undefined case
Pf(A) = 0.
"""
from __future__ import annotations

import math

import numpy as np
import pytest


def _skew_int(n, rng):
    X = rng.integers(-4, 5, size=(n, n)).astype(np.float64)
    return np.tril(X, -1) - np.tril(X, -1).T


@pytest.mark.parametrize("n,r", [(2, 1), (4, 1), (4, 2), (6, 1), (6, 2), (8, 3), (10, 2)])
def test_ratio_bruteforce(oracle_mod, n, r):
    rng = np.random.default_rng(100 * n + r)
    for _ in range(3):
        A = _skew_int(n, rng)
        U = rng.integers(-2, 3, size=(n, r)).astype(np.float64)
        V = rng.integers(-2, 3, size=(n, r)).astype(np.float64)
        B = A + U @ V.T - V @ U.T
        pa = oracle_mod.pfaffian_bruteforce(A)
        pb = oracle_mod.pfaffian_bruteforce(B)
        la, s, info = oracle_mod.pf_ratio(A, U, V)
        if pa == 0:
            assert info > 0 and s == 0 and math.isnan(la)
            continue
        exact = pb / pa
        assert info == 0
        if exact == 0:
            assert s == 0 and la == -math.inf
        else:
            assert s == (1 if exact > 0 else -1)
            assert abs(la - math.log(abs(float(exact)))) <= 1e-12 * max(1.0, abs(la))


def test_ratio_block_diagonal_closed_form(oracle_mod):
    # blocks [[0, -d_i], [d_i, 0]] (lower entry d_i); U = t e_0, V = e_1 changes the
    # lower entry of block 0 to d_0 - t, so the ratio is (d_0 - t) / d_0
    n = 40
    d = np.linspace(0.5, 3.0, n // 2) * np.where(np.arange(n // 2) % 2 == 0, 1.0, -1.0)
    A = np.zeros((n, n))
    for i in range(n // 2):
        A[2 * i + 1, 2 * i], A[2 * i, 2 * i + 1] = d[i], -d[i]
    for t in (0.25, 2.0, -1.5):
        U = np.zeros((n, 1))
        V = np.zeros((n, 1))
        U[0, 0], V[1, 0] = t, 1.0
        la, s, info = oracle_mod.pf_ratio(A, U, V)
        want = (d[0] - t) / d[0]
        assert info == 0 and s == np.sign(want)
        assert abs(la - math.log(abs(want))) <= 1e-14


def test_ratio_no_change_and_composition(oracle_mod, gen):
    n = 60
    A = gen.skew_gaussian(n, 3)
    rng = np.random.default_rng(7)
    U = rng.standard_normal((n, 3))
    la, s, info = oracle_mod.pf_ratio(A, U, U)   # U V^T - V U^T = 0
    assert info == 0 and s == 1 and la == 0.0
    U1, V1 = rng.standard_normal((n, 2)), rng.standard_normal((n, 2))
    U2, V2 = rng.standard_normal((n, 1)), rng.standard_normal((n, 1))
    S = oracle_mod.full_from_lower(A)
    B1 = S + (U1 @ V1.T - V1 @ U1.T)
    la1, s1, _ = oracle_mod.pf_ratio(A, U1, V1)
    la2, s2, _ = oracle_mod.pf_ratio(B1, U2, V2)
    la12, s12, _ = oracle_mod.pf_ratio(A, np.hstack([U1, U2]), np.hstack([V1, V2]))
    assert s1 * s2 == s12 and abs(la1 + la2 - la12) <= 1e-12 * max(1.0, abs(la12))


def test_ratio_undefined_when_pf_a_is_zero(oracle_mod, gen):
    A = gen.skew_gaussian(7, 1)                  # odd order: Pf(A) = 0
    la, s, info = oracle_mod.pf_ratio(A, np.ones((7, 1)), np.arange(7.0).reshape(7, 1))
    assert math.isnan(la) and s == 0 and info == 7
    Z = gen.skew_gaussian(10, 2).copy()
    Z[:, 4] = 0.0
    Z[4, :] = 0.0
    la, s, info = oracle_mod.pf_ratio(Z, np.ones((10, 1)), np.arange(10.0).reshape(10, 1))
    assert math.isnan(la) and s == 0 and info > 0
