"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test fixes the oracle's output by an independent route: a hand-derived
example, exact brute-force Pfaffians, LAPACK's LU determinant, closed forms,
algebraic identities and structural invariants.  A plausible slip in the oracle
(a dropped term, a wrong sign in the skew interchange, a transposed operand, a
wrong tie-break, a wrong swap count) fails at least one of them.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _skew_from_upper(n, rng, lo=-3, hi=3):
    A = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            v = float(rng.integers(lo, hi + 1))
            A[i, j] = v
            A[j, i] = -v
    return A


def _pf_value(la, s):
    return 0.0 if s == 0 else s * math.exp(la)


def _read_worked():
    path = os.path.join(HERE, "golden", "worked_4x4.txt")
    d = {"upper": [], "L": []}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        if key in ("upper", "L"):
            d[key].append(vals)
        else:
            d[key] = vals
    return d


def test_worked_4x4_example(oracle_mod):
    d = _read_worked()
    n = int(d["n"][0])
    A = np.zeros((n, n))
    for i, j, v in d["upper"]:
        i, j, v = int(i), int(j), float(Fraction(v))
        A[i, j], A[j, i] = v, -v
    f = oracle_mod.ltlt(A)
    assert f.info == 0
    assert f.ipiv.tolist() == [int(x) for x in d["ipiv"]]
    np.testing.assert_allclose(f.T, [float(Fraction(x)) for x in d["T"]], rtol=1e-15, atol=0)
    for i, j, v in d["L"]:
        i, j = int(i), int(j)
        assert abs(f.LT[i, j - 1] - float(Fraction(v))) <= 1e-15
    la, s = oracle_mod.logpf_from_factors(n, f.ipiv, f.T)
    assert s == 1 and abs(math.exp(la) - float(Fraction(d["pfaffian"][0]))) < 1e-13
    assert oracle_mod.pfaffian_bruteforce(A) == Fraction(d["pfaffian"][0])


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_bruteforce_small_integer(oracle_mod, n):
    rng = np.random.default_rng(100 + n)
    for trial in range(6):
        A = _skew_from_upper(n, rng)
        exact = oracle_mod.pfaffian_bruteforce(A)
        la, s, info = oracle_mod.logpf(A)
        got = _pf_value(la, s)
        if n % 2 == 1:
            assert exact == 0 and s == 0
            continue
        if exact == 0:
            # exactly singular even matrix: rounding may leave a tiny pivot
            assert abs(got) <= 1e-9 * max(1.0, np.abs(A).max()) ** (n // 2)
        else:
            assert abs(got - float(exact)) <= 1e-12 * abs(float(exact)), (n, trial, got, exact)


def test_bruteforce_sign_count_with_many_swaps(oracle_mod):
    # magnitudes increasing down each column force an interchange at every step
    n = 8
    A = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            v = float((j + 1) ** 2 + i) * (1 if (i + j) % 3 else -1)
            A[i, j], A[j, i] = v, -v
    f = oracle_mod.ltlt(A)
    assert (f.ipiv[1:] != np.arange(1, n)).sum() >= 3
    la, s = oracle_mod.logpf_from_factors(n, f.ipiv, f.T)
    exact = float(oracle_mod.pfaffian_bruteforce(A))
    assert abs(_pf_value(la, s) - exact) <= 1e-12 * abs(exact)


@pytest.mark.parametrize("n", [2, 8, 64, 256, 512])
def test_pf_squared_equals_det(oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 11 + n)
    la, s, info = oracle_mod.logpf(A)
    assert info == 0 and s in (-1, 1)
    dsign, dlog = oracle_mod.logdet_lu(A)
    assert dsign == 1.0
    assert abs(2 * la - dlog) <= 1e-12 * max(1.0, abs(dlog)) * max(1.0, n / 64)


@pytest.mark.parametrize("n", [2, 6, 40, 200])
def test_block_diagonal_permuted(oracle_mod, n):
    rng = np.random.default_rng(7 * n)
    d = rng.uniform(0.5, 2.0, n // 2) * rng.choice([-1.0, 1.0], n // 2)
    J = np.zeros((n, n))
    for i in range(n // 2):
        J[2 * i, 2 * i + 1], J[2 * i + 1, 2 * i] = d[i], -d[i]
    perm = rng.permutation(n)
    Q = np.eye(n)[perm]
    A = Q @ J @ Q.T
    # det(Q) of a permutation matrix: parity of the permutation
    seen, parity = np.zeros(n, bool), 0
    for i in range(n):
        if not seen[i]:
            j, ln = i, 0
            while not seen[j]:
                seen[j], j, ln = True, perm[j], ln + 1
            parity ^= (ln - 1) & 1
    detQ = -1 if parity else 1
    la, s, info = oracle_mod.logpf(A)
    assert info == 0
    assert s == detQ * int(np.sign(np.prod(d)))
    assert abs(la - np.log(np.abs(d)).sum()) <= 1e-13 * max(1, n)


@pytest.mark.parametrize("n", [4, 32, 128])
def test_congruence_known_pf(oracle_mod, n):
    rng = np.random.default_rng(3 * n)
    d = rng.uniform(0.5, 2.0, n // 2)
    J = np.zeros((n, n))
    for i in range(n // 2):
        J[2 * i, 2 * i + 1], J[2 * i + 1, 2 * i] = d[i], -d[i]
    B = np.tril(rng.standard_normal((n, n)) * 0.3, -1) + np.diag(rng.uniform(0.5, 2.0, n))
    A = B @ J @ B.T
    A = 0.5 * (A - A.T)
    la, s, info = oracle_mod.logpf(A)
    expect = np.log(np.diag(B)).sum() + np.log(d).sum()
    assert info == 0 and s == 1
    assert abs(la - expect) <= 1e-11 * max(1.0, abs(expect))


@pytest.mark.parametrize("m", [1, 2, 3, 5, 16])
def test_off_diagonal_block(oracle_mod, m):
    rng = np.random.default_rng(m)
    M = rng.standard_normal((m, m))
    n = 2 * m
    A = np.zeros((n, n))
    A[:m, m:] = M
    A[m:, :m] = -M.T
    la, s, info = oracle_mod.logpf(A)
    ds, dl = np.linalg.slogdet(M)
    expect_sign = int(ds) * (-1 if (m * (m - 1) // 2) % 2 else 1)
    assert s == expect_sign
    assert abs(la - dl) <= 1e-12 * max(1.0, abs(dl))


@pytest.mark.parametrize("n", [6, 50])
def test_scaling_and_transpose(oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 5 + n)
    la, s, _ = oracle_mod.logpf(A)
    la2, s2, _ = oracle_mod.logpf(4.0 * A)         # Pf(cA) = c^{n/2} Pf(A), exact for c = 4
    assert s2 == s and abs(la2 - (la + (n // 2) * math.log(4.0))) <= 1e-12 * max(1, abs(la2))
    la3, s3, _ = oracle_mod.logpf(np.ascontiguousarray(A.T))  # Pf(A^T) = (-1)^{n/2} Pf(A)
    assert s3 == s * (-1) ** (n // 2) and abs(la3 - la) <= 1e-12 * max(1, abs(la))


@pytest.mark.parametrize("n", [3, 17, 64, 255, 512])
def test_factor_invariants_and_reconstruction(oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 1000 + n)
    f = oracle_mod.ltlt(A)
    assert f.info == 0
    assert f.ipiv[0] == 0 and all(f.ipiv[j] >= j for j in range(n))
    if n >= 2:
        assert f.ipiv[n - 1] == n - 1
    L, Tm, perm = oracle_mod.reconstruct(f.LT, f.ipiv, f.T)
    assert np.abs(np.tril(L, -1)).max() <= 1.0
    assert oracle_mod.recon_residual(A, f.LT, f.ipiv, f.T) <= 1e-15
    # upper triangle and diagonal are never written
    assert np.array_equal(np.triu(f.LT), np.triu(A))


def test_only_lower_triangle_read(oracle_mod, gen):
    n = 40
    A = gen.skew_gaussian(n, 77)
    B = A.copy()
    B[np.triu_indices(n)] = np.nan          # garbage above and on the diagonal
    fa, fb = oracle_mod.ltlt(A), oracle_mod.ltlt(B)
    assert fb.info == 0
    assert np.array_equal(fa.ipiv, fb.ipiv) and np.array_equal(fa.T, fb.T)
    assert np.array_equal(np.tril(fa.LT, -1), np.tril(fb.LT, -1))


def test_tie_break_lowest_index(oracle_mod):
    n = 6
    A = np.zeros((n, n))
    # column 0 below the diagonal: |.| = (1, 3, 3, 2, 3) -> first maximum is row 2
    col = [1.0, -3.0, 3.0, 2.0, -3.0]
    for i, v in enumerate(col, start=1):
        A[i, 0], A[0, i] = v, -v
    rng = np.random.default_rng(0)
    for i in range(1, n):
        for j in range(1, i):
            v = float(rng.integers(-2, 3))
            A[i, j], A[j, i] = v, -v
    f = oracle_mod.ltlt(A)
    assert f.ipiv[1] == 2


def test_zero_column_gives_zero_pivot(oracle_mod, gen):
    n = 10
    A = gen.skew_gaussian(n, 9)
    A[:, 0] = 0.0
    A[0, :] = 0.0
    f = oracle_mod.ltlt(A)
    assert f.T[0] == 0.0 and f.ipiv[1] == 1 and f.info == 1
    assert np.all(f.LT[2:, 0] == 0.0)
    la, s = oracle_mod.logpf_from_factors(n, f.ipiv, f.T)
    assert s == 0 and la == -math.inf
    assert oracle_mod.pfaffian_bruteforce(np.round(A * 0)) == 0


def test_nonfinite_reported(oracle_mod, gen):
    A = gen.skew_gaussian(12, 4)
    A[7, 0] = np.nan
    assert oracle_mod.ltlt(A).info == oracle_mod.ENONFINITE
    A = gen.skew_gaussian(12, 4)
    A[9, 5] = np.inf
    assert oracle_mod.ltlt(A).info == oracle_mod.ENONFINITE


@pytest.mark.parametrize("n,nrhs", [(2, 1), (8, 3), (64, 16), (300, 5)])
def test_solve_backward_error(oracle_mod, gen, n, nrhs):
    A = gen.skew_gaussian(n, 200 + n)
    B = gen.gaussian(n, nrhs, 300 + n)
    f = oracle_mod.ltlt(A)
    X, info = oracle_mod.solve(f.LT, f.ipiv, f.T, B)
    assert info == 0
    assert oracle_mod.backward_error(A, X, B) <= 1e-14
    # against an independent LU solve of the full matrix
    Xr = np.linalg.solve(oracle_mod.full_from_lower(A), B)
    assert np.abs(X - Xr).max() <= 1e-8 * np.abs(Xr).max() * n


def test_solve_singular(oracle_mod, gen):
    A = gen.skew_gaussian(7, 1)
    f = oracle_mod.ltlt(A)
    _, info = oracle_mod.solve(f.LT, f.ipiv, f.T, np.ones((7, 1)))
    assert info == 7


def test_skr2k_oracle_against_exact_integers(oracle_mod):
    rng = np.random.default_rng(5)
    n, k = 7, 3
    A = rng.integers(-4, 5, (n, k)).astype(float)
    B = rng.integers(-4, 5, (n, k)).astype(float)
    C = rng.integers(-4, 5, (n, n)).astype(float)
    alpha, beta = 2.0, -1.0
    out = oracle_mod.skr2k(alpha, A, B, beta, C)
    for i in range(n):
        for j in range(n):
            if i > j:
                s = sum(int(A[i, q]) * int(B[j, q]) - int(B[i, q]) * int(A[j, q]) for q in range(k))
                assert out[i, j] == beta * C[i, j] + alpha * s
            else:
                assert out[i, j] == C[i, j]
    # A = B gives a zero update exactly; the bound is zero for zero inputs
    assert np.array_equal(oracle_mod.skr2k(1.0, A, A, 1.0, C), C)
    assert not oracle_mod.skr2k_error_bound(1.0, 0 * A, 0 * B, 0.0, C).any()


def test_generator_log_and_moments(gen):
    for x in [1e-300, 1e-5, 0.1, 0.5, 0.70710678, 0.75, 0.999999, 1.0, 2.0, 12345.678]:
        assert abs(gen.log(x) - math.log(x)) <= 4 * np.spacing(abs(math.log(x)) + 1e-300) + 1e-300
    z = np.array([gen.gauss(3, 9, c) for c in range(20000)])
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1.0) < 0.04
    A = gen.skew_gaussian(33, 8)
    assert np.array_equal(A, -A.T) and not np.diag(A).any()
    sizes = gen.even_sizes(5000, 32, 512, 7)
    assert sizes.min() >= 32 and sizes.max() <= 512 and np.all(sizes % 2 == 0)


def test_generator_golden_hash(gen):
    import hashlib
    A = gen.skew_gaussian(64, 1)
    h = hashlib.sha256(np.asfortranarray(A).tobytes(order="F")).hexdigest()
    ref = open(os.path.join(HERE, "golden", "skew_gaussian_n64_s1.sha256")).read().split()[0]
    assert h == ref
    # threaded and single-threaded fills agree bit for bit
    big1 = gen.skew_gaussian(600, 3, threads=1)
    big8 = gen.skew_gaussian(600, 3, threads=8)
    assert np.array_equal(big1, big8)


@pytest.mark.parametrize("n,seed", [(50, 1), (300, 2), (1000, 3)])
def test_designed_exact_ties(oracle_mod, n, seed):
    """A matrix with a known factorization, exact ties at nearly every step
    (spread over the whole column) and exact arithmetic: the oracle must return
    the designed interchanges (ties to the lowest index), T0 and L0 bit for bit."""
    from designed_ties import designed
    A, ipiv, T0, L0 = designed(n, seed)
    f = oracle_mod.ltlt(A, nthreads=4)
    assert f.info == 0
    assert np.array_equal(f.ipiv, ipiv)
    assert np.array_equal(f.T, T0)
    for j in range(1, n - 1):
        assert np.array_equal(f.LT[j + 1:, j - 1], L0[j + 1:, j]), j
    assert np.count_nonzero(f.gap == 0.0) > n // 2            # exact ties at most steps
    assert np.count_nonzero(ipiv != np.arange(n)) >= n // 20  # and interchanges
