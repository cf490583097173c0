"""Pins of the oracle's magnitude sums, which set the per-entry tolerance of T
and L in the parity tests (the summation-error bound gamma_m * sum |terms|).

They are fixed by a hand-derived example, by exact rational elimination along
the oracle's own pivots (the bound must hold for the oracle's evaluation), by
structure (no updates: the sums are the inputs' magnitudes) and by scaling
(every term scales with the matrix).
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _worked():
    d = {"upper": []}
    for line in open(os.path.join(HERE, "golden", "worked_4x4.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        if key == "upper":
            d["upper"].append(vals)
        else:
            d[key] = vals
    n = int(d["n"][0])
    A = np.zeros((n, n))
    for i, j, v in d["upper"]:
        A[int(i), int(j)], A[int(j), int(i)] = float(Fraction(v)), -float(Fraction(v))
    return A, [float(Fraction(x)) for x in d["Tmag"]]


def test_worked_example_magnitudes(oracle_mod):
    A, tmag = _worked()
    f = oracle_mod.ltlt(A, want_mag=True)
    np.testing.assert_allclose(f.T_mag(), tmag, rtol=1e-15, atol=0)
    # the Pfaffian-only mode takes the same step 0 and then stops at T[2]
    ipiv, T, info, Tm = oracle_mod.pfonly(A, want_mag=True)
    np.testing.assert_allclose(Tm, [tmag[0], 0.0, tmag[2]], rtol=1e-15, atol=0)


def _exact_elimination(A, ipiv, step):
    """T by exact rational elimination along the given interchanges."""
    n = A.shape[0]
    S = [[Fraction(float(A[i, j])) - Fraction(float(A[j, i])) if i > j else Fraction(0)
          for j in range(n)] for i in range(n)]
    W = [[Fraction(0)] * n for _ in range(n)]  # full skew copy
    for i in range(n):
        for j in range(i):
            W[i][j], W[j][i] = S[i][j] / 2, -S[i][j] / 2
    T = [Fraction(0)] * max(n - 1, 0)
    for k in range(0, n - 2, step):
        r, p = k + 1, int(ipiv[k + 1])
        W[r], W[p] = W[p], W[r]
        for row in W:
            row[r], row[p] = row[p], row[r]
        a = W[k + 1][k]
        T[k] = a
        l = [W[i][k] / a if a != 0 else Fraction(0) for i in range(n)]
        v = [W[i][k + 1] for i in range(n)]
        for i in range(k + 2, n):
            for j in range(k + 2, n):
                W[i][j] += l[i] * v[j] - v[i] * l[j]
    if n >= 2:
        T[n - 2] = W[n - 1][n - 2]
    return T


@pytest.mark.parametrize("n", [6, 9, 12, 15])
def test_bound_holds_against_exact_arithmetic(oracle_mod, gen, n):
    # Gaussian input with entries rounded to 20 bits: exact in binary, so the
    # rational elimination starts from exactly the oracle's input
    A = np.round(gen.skew_gaussian(n, 70 + n) * 2 ** 20) / 2 ** 20
    A = np.tril(A, -1) - np.tril(A, -1).T
    f = oracle_mod.ltlt(A, want_mag=True)
    Tx = _exact_elimination(A, f.ipiv, 1)
    err = np.array([abs(Fraction(float(t)) - x) for t, x in zip(f.T, Tx)], dtype=np.float64)
    k = np.arange(n - 1)
    bound = oracle_mod.gamma(2 * k + 1) * f.T_mag()
    assert np.all(err <= bound), (err, bound)
    assert np.all(f.T_mag() >= np.abs(f.T))
    if n % 2 == 1:
        return  # the Pfaffian-only reduction does no work for odd n
    ipiv, T, info, Tm = oracle_mod.pfonly(A, want_mag=True)
    Tx = _exact_elimination(A, ipiv, 2)
    for kk in range(0, n - 1, 2):
        e = abs(Fraction(float(T[kk])) - Tx[kk])
        assert float(e) <= oracle_mod.gamma(kk + 1) * Tm[kk], (kk, float(e), Tm[kk])


@pytest.mark.parametrize("n", [4, 10, 64])
def test_no_updates_give_input_magnitudes(oracle_mod, n):
    rng = np.random.default_rng(n)
    d = rng.uniform(0.5, 2.0, n // 2) * rng.choice([-1.0, 1.0], n // 2)
    A = np.zeros((n, n))
    for i in range(n // 2):
        A[2 * i + 1, 2 * i], A[2 * i, 2 * i + 1] = -d[i], d[i]
    f = oracle_mod.ltlt(A, want_mag=True)
    np.testing.assert_array_equal(f.T_mag(), np.abs(f.T))
    assert np.array_equal(f.T_mag()[0::2], np.abs(d))


@pytest.mark.parametrize("n", [7, 33, 128])
def test_magnitudes_scale_with_the_matrix(oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 90 + n)
    f1 = oracle_mod.ltlt(A, want_mag=True)
    f2 = oracle_mod.ltlt(A * 8.0, want_mag=True)
    assert np.array_equal(f1.ipiv, f2.ipiv)
    low = np.tril(np.ones((n, n), bool), -1)
    np.testing.assert_array_equal(f2.M[low], 8.0 * f1.M[low])
    _, _, _, m1 = oracle_mod.pfonly(A, want_mag=True)
    _, _, _, m2 = oracle_mod.pfonly(A * 0.25, want_mag=True)
    np.testing.assert_array_equal(m2, 0.25 * m1)
