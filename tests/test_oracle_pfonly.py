"""Pins of the oracle's Pfaffian-only reduction (elimination at even steps only).

Its pivot sequence differs from the full factorization's, so it is pinned on
its own: the hand-derived 4x4 example (tests/golden/worked_4x4.txt, whose
factorization has no odd-step interchange, so the even steps coincide with the
full ones), exact brute-force Pfaffians, LAPACK's LU determinant, the block
diagonal closed form under a random permutation, the tie-break, zero and
non-finite columns, and agreement with the full factorization's Pfaffian.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np
import pytest

from test_oracle_pins import _pf_value, _read_worked, _skew_from_upper


def test_pfonly_worked_4x4(oracle_mod):
    d = _read_worked()
    n = int(d["n"][0])
    A = np.zeros((n, n))
    for i, j, v in d["upper"]:
        i, j, v = int(i), int(j), float(Fraction(v))
        A[i, j], A[j, i] = v, -v
    ipiv, T, info = oracle_mod.pfonly(A)
    assert info == 0
    assert ipiv.tolist() == [int(x) for x in d["ipiv"]]
    Tf = [float(Fraction(x)) for x in d["T"]]
    assert T[0] == Tf[0] and abs(T[2] - Tf[2]) <= 1e-15 and T[1] == 0.0
    la, s, _ = oracle_mod.logpf_pfonly(A)
    assert s == 1 and abs(math.exp(la) - float(Fraction(d["pfaffian"][0]))) < 1e-13


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_pfonly_bruteforce_small_integer(oracle_mod, n):
    rng = np.random.default_rng(300 + n)
    for trial in range(6):
        A = _skew_from_upper(n, rng)
        exact = oracle_mod.pfaffian_bruteforce(A)
        la, s, info = oracle_mod.logpf_pfonly(A)
        got = _pf_value(la, s)
        if n % 2 == 1:
            assert exact == 0 and s == 0 and info == n
            continue
        if exact == 0:
            assert abs(got) <= 1e-9 * max(1.0, np.abs(A).max()) ** (n // 2)
        else:
            assert abs(got - float(exact)) <= 1e-12 * abs(float(exact)), (n, trial, got, exact)


def test_pfonly_many_swaps(oracle_mod):
    n = 10
    A = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            v = float((j + 1) ** 2 + i) * (1 if (i + j) % 3 else -1)
            A[i, j], A[j, i] = v, -v
    ipiv, T, info = oracle_mod.pfonly(A)
    assert info == 0
    assert all(ipiv[j] == j for j in range(0, n, 2))          # only odd positions interchange
    assert (ipiv != np.arange(n)).sum() >= 2
    la, s = oracle_mod.logpf_from_factors(n, ipiv, T)
    exact = float(oracle_mod.pfaffian_bruteforce(A))
    assert abs(_pf_value(la, s) - exact) <= 1e-12 * abs(exact)


@pytest.mark.parametrize("n", [2, 8, 64, 256])
def test_pfonly_squared_equals_det(oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 21 + n)
    la, s, info = oracle_mod.logpf_pfonly(A)
    assert info == 0 and s in (-1, 1)
    dsign, dlog = oracle_mod.logdet_lu(A)
    assert dsign == 1.0
    assert abs(2 * la - dlog) <= 1e-12 * max(1.0, abs(dlog)) * max(1.0, n / 64)


@pytest.mark.parametrize("n", [2, 6, 40, 200])
def test_pfonly_block_diagonal_permuted(oracle_mod, n):
    rng = np.random.default_rng(11 * n)
    d = rng.uniform(0.5, 2.0, n // 2) * rng.choice([-1.0, 1.0], n // 2)
    J = np.zeros((n, n))
    for i in range(n // 2):
        J[2 * i, 2 * i + 1], J[2 * i + 1, 2 * i] = d[i], -d[i]
    perm = rng.permutation(n)
    Q = np.eye(n)[perm]
    A = Q @ J @ Q.T
    seen, parity = np.zeros(n, bool), 0
    for i in range(n):
        if not seen[i]:
            j, ln = i, 0
            while not seen[j]:
                seen[j], j, ln = True, perm[j], ln + 1
            parity ^= (ln - 1) & 1
    la, s, info = oracle_mod.logpf_pfonly(A)
    assert info == 0
    assert s == (-1 if parity else 1) * int(np.sign(np.prod(d)))
    assert abs(la - np.log(np.abs(d)).sum()) <= 1e-13 * max(1, n)


@pytest.mark.parametrize("n", [50, 128, 300])
def test_pfonly_agrees_with_full_factorization(oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 40 + n)
    la1, s1, i1 = oracle_mod.logpf_pfonly(A)
    la2, s2, i2 = oracle_mod.logpf(A)
    assert i1 == 0 and i2 == 0 and s1 == s2
    assert abs(la1 - la2) <= 1e-12 * max(1.0, abs(la2))


def test_pfonly_tie_break_and_zero_column(oracle_mod):
    # column 0 holds +2 at rows 2 and 3 and -2 at row 1: equal magnitudes -> row 1 (no swap)
    n = 4
    A = np.zeros((n, n))
    A[1, 0], A[2, 0], A[3, 0] = -2.0, 2.0, 2.0
    A[2, 1], A[3, 1], A[3, 2] = 1.0, 3.0, 5.0
    A = np.tril(A, -1) - np.tril(A, -1).T
    ipiv, T, info = oracle_mod.pfonly(A)
    assert ipiv[1] == 1 and T[0] == -2.0
    # an all-zero first column: zero pivot, no interchange, singular
    B = np.array(A)
    B[:, 0] = 0.0
    B[0, :] = 0.0
    ipiv, T, info = oracle_mod.pfonly(B)
    assert info == 1 and ipiv[1] == 1 and T[0] == 0.0
    la, s, _ = oracle_mod.logpf_pfonly(B)
    assert s == 0 and la == -math.inf


def test_pfonly_nonfinite_reported(oracle_mod, gen):
    A = gen.skew_gaussian(16, 5)
    A[9, 2], A[2, 9] = np.nan, np.nan
    ipiv, T, info = oracle_mod.pfonly(A)
    assert info == oracle_mod.ENONFINITE
