"""Pins of the oracle's complex (complex128) LTL^T and of the solve with its
factors.

* Real input: the complex factorization is the real C oracle's bit for bit
  (interchanges, T and L) and so is the solve (every complex operation with
  zero imaginary parts is the real one; the division is Smith's with true
  divisions).
* Reconstruction P A P^T = L T L^T, L unit lower with |L| <= 1, T skew
  tridiagonal, to rounding, on Gaussian and Gaussian-integer matrices.
* The Pfaffian from the factors against exact brute-force Pfaffians (n <= 10)
  and against the Pfaffian-only reduction, a different elimination order.
* Conjugation: conj(A) gives the conjugate factors with the same interchanges.
* The solve: backward error with the original matrix, odd order and a zero
  pivot reported as for real input, a closed-form block-diagonal system.
"""
from __future__ import annotations

import math

import numpy as np
import pytest


def _cgauss(n, rng):
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return np.tril(X, -1) - np.tril(X, -1).T


def _cint(n, rng, r=3):
    X = rng.integers(-r, r + 1, size=(n, n)) + 1j * rng.integers(-r, r + 1, size=(n, n))
    return np.tril(X, -1) - np.tril(X, -1).T


def _parts(LT, ip, T):
    n = LT.shape[0]
    L = np.eye(n, dtype=np.complex128)
    if n > 1:
        L[:, 1:] += np.tril(LT, -2)[:, :-1]
    Tm = np.diag(T, -1) - np.diag(T, 1) if n > 1 else np.zeros((n, n), dtype=np.complex128)
    P = np.eye(n)
    for j in range(1, n):
        if ip[j] != j:
            P[[j, ip[j]]] = P[[ip[j], j]]
    return L, Tm, P


@pytest.mark.parametrize("n", [40, 41, 97])
def test_real_input_is_the_real_oracle(oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 70 + n)
    f = oracle_mod.ltlt(A)
    LT, ip, T, info = oracle_mod.ltlt_c128(A)
    assert info == f.info and np.array_equal(ip, f.ipiv)
    assert np.array_equal(T.real, f.T) and not np.any(T.imag)
    assert np.array_equal(np.tril(LT.real, -2), np.tril(f.LT, -2)) and not np.any(LT.imag)
    B = gen.gaussian(n, 3, 71 + n)
    X, i1 = oracle_mod.solve(f.LT, f.ipiv, f.T, B)
    Xc, i2 = oracle_mod.solve_c128(LT, ip, T, B)
    assert i1 == i2 and np.array_equal(Xc.real, X) and not np.any(Xc.imag)


@pytest.mark.parametrize("n", [2, 3, 4, 7, 16, 33, 64])
def test_reconstruction(oracle_mod, n):
    rng = np.random.default_rng(900 + n)
    for A in (_cgauss(n, rng), _cint(n, rng)):
        LT, ip, T, info = oracle_mod.ltlt_c128(A)
        L, Tm, P = _parts(LT, ip, T)
        assert np.all(np.abs(L) <= 1.0 + 1e-15)
        assert np.all(ip[1:] >= np.arange(1, n)) and ip[0] == 0
        R = P @ A @ P.T - L @ Tm @ L.T
        assert np.abs(R).max() <= 64 * n * 2.0 ** -53 * max(1.0, np.abs(A).max()) * n, np.abs(R).max()


@pytest.mark.parametrize("n", [2, 4, 6, 8, 10])
def test_pfaffian_bruteforce(oracle_mod, n):
    rng = np.random.default_rng(1700 + n)
    for _ in range(3):
        A = _cint(n, rng)
        exact = oracle_mod.pfaffian_bruteforce_complex(A)
        LT, ip, T, info = oracle_mod.ltlt_c128(A)
        la, ph = oracle_mod.logpf_c128_from_factors(n, ip, T)
        if exact == 0:
            assert ph == 0 and la == -math.inf
            continue
        got = math.exp(la) * ph
        assert abs(got - exact) <= 1e-10 * abs(exact), (got, exact)


def test_pfaffian_against_pfonly_and_conjugation(oracle_mod):
    rng = np.random.default_rng(5)
    n = 64
    A = _cgauss(n, rng)
    LT, ip, T, info = oracle_mod.ltlt_c128(A)
    la, ph = oracle_mod.logpf_c128_from_factors(n, ip, T)
    ip2, T2, info2 = oracle_mod.pfonly_c128(A)
    la2, ph2 = oracle_mod.logpf_c128_from_factors(n, ip2, T2)
    assert info == info2 == 0
    assert abs(la - la2) <= 1e-12 * abs(la) and abs(ph - ph2) <= 1e-11
    LTc, ipc, Tc, infoc = oracle_mod.ltlt_c128(np.conj(A))
    assert np.array_equal(ipc, ip) and np.array_equal(Tc, np.conj(T)) and np.array_equal(LTc, np.conj(LT))


def test_magnitude_sums(oracle_mod):
    """M[k+1, k] bounds |T[k]| and M[i, j-1] bounds |L[i, j] T[j-1]| (a sum is at
    most the sum of its terms' magnitudes, to rounding); on real input they are
    the real oracle's."""
    rng = np.random.default_rng(8)
    n = 50
    A = _cgauss(n, rng)
    LT, ip, T, info, M = oracle_mod.ltlt_c128(A, want_mag=True)
    Tm = np.array([M[k + 1, k] for k in range(n - 1)])
    assert np.all(np.abs(T) <= Tm * (1 + 1e-12))
    for j in range(1, n - 1):
        num = np.abs(LT[j + 1:, j - 1] * T[j - 1])
        assert np.all(num <= M[j + 1:, j - 1] * (1 + 1e-12) + 1e-300)
    R = np.tril(rng.standard_normal((n, n)), -1)
    f = oracle_mod.ltlt(R, want_mag=True)
    *_, Mc = oracle_mod.ltlt_c128(R, want_mag=True)
    assert np.allclose(np.tril(Mc, -1), np.tril(f.M, -1), rtol=1e-13, atol=0)


def test_solve(oracle_mod):
    rng = np.random.default_rng(11)
    for n in (2, 4, 30, 64):
        A = _cgauss(n, rng)
        B = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
        LT, ip, T, info = oracle_mod.ltlt_c128(A)
        X, inf2 = oracle_mod.solve_c128(LT, ip, T, B)
        assert info == inf2 == 0
        r = np.abs(A @ X - B).max(axis=0)
        eta = r / (np.abs(A).sum(1).max() * np.abs(X).max(axis=0) + np.abs(B).max(axis=0))
        assert eta.max() <= 1e-14, eta
    # block diagonal: A = diag([[0, -d_i], [d_i, 0]]), x_{2i} = b_{2i+1}/d_i, x_{2i+1} = -b_{2i}/d_i
    m = 6
    d = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    A = np.zeros((2 * m, 2 * m), dtype=np.complex128)
    for i in range(m):
        A[2 * i + 1, 2 * i], A[2 * i, 2 * i + 1] = d[i], -d[i]
    b = rng.standard_normal(2 * m) + 1j * rng.standard_normal(2 * m)
    X, inf3 = oracle_mod.solve_c128(*oracle_mod.ltlt_c128(A)[:3], b)
    want = np.empty(2 * m, dtype=np.complex128)
    want[0::2], want[1::2] = b[1::2] / d, -b[0::2] / d
    assert inf3 == 0 and np.abs(X[:, 0] - want).max() <= 1e-14 * np.abs(want).max()
    # odd order, zero pivot
    A7 = _cgauss(7, rng)
    assert oracle_mod.solve_c128(*oracle_mod.ltlt_c128(A7)[:3], np.ones(7))[1] == 7
    Z = _cgauss(10, rng)
    Z[:, 0] = 0
    Z[0, :] = 0
    LT, ip, T, info = oracle_mod.ltlt_c128(Z)
    assert info == 1 and oracle_mod.solve_c128(LT, ip, T, np.ones(10))[1] == 1
