"""Pins of the oracle's complex (complex128) Pfaffian-only reduction.

Exact brute-force Pfaffians on Gaussian-integer matrices (n <= 10), Pf^2 = det
against LAPACK's complex LU determinant, a real matrix giving the real
oracle's interchanges and pivots, the block-diagonal closed form under a
random symmetric permutation, the scaling identity Pf(c A) = c^{n/2} Pf(A),
odd order, a zero row and a non-finite entry.
"""
from __future__ import annotations

import math

import numpy as np
import pytest


def _skew_cint(n, rng, r=3):
    X = rng.integers(-r, r + 1, size=(n, n)) + 1j * rng.integers(-r, r + 1, size=(n, n))
    return np.tril(X, -1) - np.tril(X, -1).T


def _pf(oracle_mod, A):
    n = A.shape[0]
    ip, T, info = oracle_mod.pfonly_c128(A)
    la, ph = oracle_mod.logpf_c128_from_factors(n, ip, T)
    return la, ph, info


@pytest.mark.parametrize("n", [0, 2, 4, 6, 8, 10])
def test_complex_bruteforce(oracle_mod, n):
    rng = np.random.default_rng(500 + n)
    for _ in range(3):
        A = _skew_cint(n, rng)
        exact = oracle_mod.pfaffian_bruteforce_complex(A)
        la, ph, info = _pf(oracle_mod, A)
        if exact == 0:
            assert ph == 0 and la == -math.inf
            continue
        assert info == 0
        got = math.exp(la) * ph
        assert abs(got - exact) <= 1e-12 * abs(exact), (n, got, exact)


@pytest.mark.parametrize("n", [12, 40, 100])
def test_complex_pf_squared_is_det(oracle_mod, n):
    rng = np.random.default_rng(600 + n)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = np.tril(X, -1) - np.tril(X, -1).T
    la, ph, info = _pf(oracle_mod, A)
    assert info == 0
    det = np.linalg.det(A)
    # log|Pf|^2 = log|det| and phase^2 = det / |det|
    assert abs(2 * la - math.log(abs(det))) <= 1e-11 * max(1.0, abs(2 * la))
    assert abs(ph * ph - det / abs(det)) <= 1e-10


def test_complex_real_input_matches_real_oracle(oracle_mod, gen):
    A = gen.skew_gaussian(64, 21)
    ip, T, info = oracle_mod.pfonly_c128(A.astype(np.complex128))
    ip_r, T_r, info_r = oracle_mod.pfonly(A)
    assert info == info_r == 0
    assert np.array_equal(ip, ip_r)
    assert np.all(T.imag == 0) and np.abs(T.real - T_r).max() <= 1e-13 * np.abs(T_r).max()


def test_complex_block_diagonal_permuted_and_scaled(oracle_mod):
    rng = np.random.default_rng(7)
    m = 12
    n = 2 * m
    d = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    B = np.zeros((n, n), dtype=np.complex128)
    for i in range(m):
        B[2 * i + 1, 2 * i], B[2 * i, 2 * i + 1] = d[i], -d[i]
    # Pf(B) = prod over blocks of B[2i, 2i+1] = prod(-d_i)
    pf_b = np.prod(-d)
    P = np.eye(n)[rng.permutation(n)]
    A = P @ B @ P.T
    # Pf(P B P^T) = det(P) Pf(B)
    want = np.linalg.det(P) * pf_b
    la, ph, info = _pf(oracle_mod, A)
    assert info == 0 and abs(math.exp(la) * ph - want) <= 1e-12 * abs(want)
    c = 0.7 - 1.3j
    la2, ph2, _ = _pf(oracle_mod, c * A)
    want2 = c ** m * want
    assert abs(math.exp(la2) * ph2 - want2) <= 1e-12 * abs(want2)


def test_complex_odd_zero_and_nonfinite(oracle_mod):
    rng = np.random.default_rng(9)
    A = _skew_cint(7, rng)
    ip, T, info = oracle_mod.pfonly_c128(A)
    assert info == 7 and np.array_equal(ip, np.arange(7)) and np.all(T == 0)
    Z = _skew_cint(10, rng)
    Z[:, 3] = 0
    Z[3, :] = 0
    la, ph, info = _pf(oracle_mod, Z)
    assert info > 0 and ph == 0 and la == -math.inf
    N = _skew_cint(10, rng).astype(np.complex128)
    N[6, 0] = complex(np.nan, 0.0)
    assert oracle_mod.pfonly_c128(N)[2] == oracle_mod.ENONFINITE


@pytest.mark.parametrize("n", [8, 64, 200])
def test_complex_magnitudes_match_real_and_rotation(oracle_mod, gen, n):
    """The magnitude sums that set the complex tolerance: for a real matrix they
    are those of the real Pfaffian-only reduction, and multiplying the matrix by
    a unit complex number leaves every magnitude unchanged."""
    R = gen.skew_gaussian(n, 400 + n)
    _, _, _, tm_real = oracle_mod.pfonly(R, want_mag=True)
    _, _, _, tm_c = oracle_mod.pfonly_c128(R.astype(np.complex128), want_mag=True)
    np.testing.assert_allclose(tm_c, tm_real, rtol=1e-13, atol=0)
    Z = R + 1j * gen.skew_gaussian(n, 500 + n)
    _, T1, _, m1 = oracle_mod.pfonly_c128(Z, want_mag=True)
    _, T2, _, m2 = oracle_mod.pfonly_c128(Z * 1j, want_mag=True)
    np.testing.assert_allclose(m2, m1, rtol=1e-13, atol=0)
    np.testing.assert_allclose(T2, 1j * T1, rtol=1e-12, atol=0)
