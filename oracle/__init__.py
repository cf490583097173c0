"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU product path never calls it.

The LTL^T factorization, the Pfaffian-only reduction (the same elimination step
at even steps only), the Pfaffian from the factors and the solve are plain C
(``ltlt_oracle.c``: the unblocked definition, FP64, no FMA contraction).  The
remaining references are written here from their definitions:

* ``pfaffian_bruteforce`` -- exact Pfaffian by expansion along the first row,
  Pf(A) = sum_{j>=1} (-1)^{j+1} a_{0j} Pf(A with rows/cols 0,j removed)
  (0-based j), in Python integers / fractions, for n <= 10;
* ``skr2k`` -- C := beta C + alpha (A B^T - B A^T) on the strict lower triangle,
  with one library matrix product per term;
* ``reconstruct`` / ``recon_residual`` -- || P A P^T - L T L^T ||_F / (n ||A||_F);
* ``backward_error`` -- max_j ||b_j - A x_j||_inf / (||A||_inf ||x_j||_inf + ||b_j||_inf);
* ``pfonly_c128`` -- the Pfaffian-only reduction of a complex skew matrix, in
  numpy complex128 on a full copy: per even step the pivot is the largest
  |z|^2 = re^2 + im^2 (each product rounded, lowest index on ties), rows and
  columns k+1 and p are interchanged, l = column k / alpha, v = column k+1, and
  l v^T - v l^T is added to the trailing block;
* ``ltlt_c128`` / ``solve_c128`` -- the LTL^T of a complex skew matrix (the real
  elimination step at every k with the complex pivot key, multipliers kept in
  place as for real input) and the solve with its factors (as the real solve,
  in complex arithmetic), in numpy complex128;
* ``pf_ratio`` -- Pf(A + U V^T - V U^T) / Pf(A) by its definition: the updated
  matrix is formed (one library product per term) and both Pfaffians are taken
  with the C factorization.

What pins the oracle (the tests under tests/test_oracle_*.py): a hand-derived
4x4 example (tests/golden/worked_4x4.txt), brute-force Pfaffians for n <= 10,
Pf(A)^2 = det(A) against LAPACK's LU determinant, closed forms for block
diagonal / congruent / off-diagonal block matrices, scaling and transposition
identities, the factor invariants (|L| <= 1, ipiv[j] >= j) and the
reconstruction residual.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ltlt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

ENONFINITE = -103


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
                               "-fno-fast-math", "-std=gnu11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            lib = ctypes.CDLL(_LIB)
            i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int32)
            lib.oracle_ltlt.restype = ctypes.c_int
            lib.oracle_ltlt.argtypes = [i64, dp, i64, ip, dp, dp, i64, ctypes.c_int]
            lib.oracle_logpf.restype = None
            lib.oracle_logpf.argtypes = [i64, ip, dp, dp, ctypes.POINTER(ctypes.c_int)]
            lib.oracle_ltlt_mag.restype = ctypes.c_int
            lib.oracle_ltlt_mag.argtypes = [i64, dp, i64, ip, dp, dp, dp, i64, i64, ctypes.c_int]
            lib.oracle_pfonly.restype = ctypes.c_int
            lib.oracle_pfonly.argtypes = [i64, dp, i64, ip, dp, ctypes.c_int]
            lib.oracle_pfonly_mag.restype = ctypes.c_int
            lib.oracle_pfonly_mag.argtypes = [i64, dp, i64, ip, dp, dp, i64, ctypes.c_int]
            lib.oracle_solve.restype = ctypes.c_int
            lib.oracle_solve.argtypes = [i64, i64, dp, i64, ip, dp, dp, i64]
            _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Factors:
    """Result of ``ltlt``: factored array (L below the subdiagonal), ipiv, T, info,
    gaps and (optionally) the per-entry magnitude sums ``M``."""

    def __init__(self, LT, ipiv, T, info, gap, M=None):
        self.LT, self.ipiv, self.T, self.info, self.gap, self.M = LT, ipiv, T, info, gap, M

    def T_mag(self) -> np.ndarray:
        """Magnitude sum of each T[k]: M[k+1, k]."""
        n = self.LT.shape[0]
        return np.array([self.M[k + 1, k] for k in range(n - 1)]) if n > 1 else np.zeros(0)


def ltlt(A: np.ndarray, nthreads: int = 1, nsteps: int = -1, want_gap: bool = True,
         inplace: bool = False, want_mag: bool = False) -> Factors:
    """Unblocked partially pivoted LTL^T of the strict lower triangle of A (FP64).

    want_mag: also return ``M`` (n x n), where M[i,j] (i > j) is the sum of the
    magnitudes of the terms entry (i,j) accumulated (the input plus |l_i v_j| +
    |v_i l_j| per update, moved with the entry by the interchanges)."""
    n = A.shape[0]
    assert A.shape == (n, n)
    LT = A if (inplace and A.flags.f_contiguous and A.dtype == np.float64) else np.array(A, dtype=np.float64, order="F")
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    T = np.zeros(max(n - 1, 1), dtype=np.float64)
    gap = np.ones(max(n, 1), dtype=np.float64) if want_gap else None
    lda = max(LT.strides[1] // 8, 1) if n > 0 else 1
    M = np.zeros((n, n), dtype=np.float64, order="F") if (want_mag and n > 0) else None
    info = _load().oracle_ltlt_mag(n, _dp(LT), lda, _ip(ipiv), _dp(T),
                                   _dp(gap) if gap is not None else None,
                                   _dp(M) if M is not None else None, max(n, 1), nsteps, nthreads)
    return Factors(LT, ipiv[:n], T[:max(n - 1, 0)], int(info),
                   gap[:max(n - 2, 0)] if gap is not None else None, M)


U_F64 = 2.0 ** -53


def gamma(m, u: float = U_F64):
    """gamma_m = m u / (1 - m u): a recursive sum of m rounded products (or m
    fused multiply-adds) differs from the exact sum by at most gamma_m times the
    sum of the magnitudes of its terms (Higham, Accuracy and Stability of
    Numerical Algorithms, section 3.1)."""
    m = np.asarray(m, dtype=np.float64)
    return m * u / (1.0 - m * u)


def t_tolerance(T_mag: np.ndarray, full: bool = True) -> np.ndarray:
    """Per-entry bound for |T_a[k] - T_b[k]| between two evaluations of the
    factorization along the same pivot sequence.  T[k] is the input entry plus
    the terms of every earlier update that reached it: at most 2k + 1 terms in
    the full factorization (2 products per step), k + 1 in the Pfaffian-only
    reduction (2 products per even step).  Each evaluation is within
    gamma_(terms + 1) * T_mag[k] of the exact sum of its terms, so the two
    differ by at most twice that."""
    k = np.arange(T_mag.size, dtype=np.float64)
    m = (2.0 * k + 2.0) if full else (k + 2.0)
    return 2.0 * gamma(m) * T_mag


def l_tolerance(L: np.ndarray, num_mag: np.ndarray, alpha: np.ndarray, alpha_mag: np.ndarray,
                col: np.ndarray) -> np.ndarray:
    """Per-entry bound for |L_a[i,j] - L_b[i,j]|: L[i,j] = c_i / alpha with the
    numerator c_i and the pivot alpha of step j-1 each within the bound of
    ``t_tolerance`` (2 gamma_(2j) times their magnitude sums), plus the rounding
    of the two divisions."""
    m = 2.0 * np.asarray(col, dtype=np.float64)
    g = 2.0 * gamma(m)
    a = np.abs(alpha)
    return (g * num_mag + np.abs(L) * g * alpha_mag) / a + 2.0 * U_F64 * np.abs(L)


def logpf_from_factors(n: int, ipiv: np.ndarray, T: np.ndarray):
    """(log|Pf|, sign) from the factors; sign 0 and -inf for a singular matrix."""
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    T = np.ascontiguousarray(T, dtype=np.float64)
    if T.size == 0:
        T = np.zeros(1)
    if ipiv.size == 0:
        ipiv = np.zeros(1, dtype=np.int32)
    la = ctypes.c_double(0.0)
    sg = ctypes.c_int(0)
    _load().oracle_logpf(n, _ip(ipiv), _dp(T), ctypes.byref(la), ctypes.byref(sg))
    return float(la.value), int(sg.value)


def logpf(A: np.ndarray, nthreads: int = 1):
    f = ltlt(A, nthreads=nthreads, want_gap=False)
    if f.info == ENONFINITE:
        return float("nan"), 0, f.info
    la, s = logpf_from_factors(A.shape[0], f.ipiv, f.T)
    return la, s, f.info


def pfonly(A: np.ndarray, nthreads: int = 1, want_mag: bool = False):
    """Pfaffian-only reduction (even elimination steps only): (ipiv, T, info),
    and with want_mag a fourth item, the magnitude sum of each T[k] (as in
    ``ltlt``; zero at the odd entries).

    ipiv[k+1] (k even) is the interchange of step k, every other ipiv[j] = j;
    T[k] (k even) are the pivots.  log|Pf| and sign follow from them exactly as
    from the full factors (``logpf_from_factors``)."""
    n = A.shape[0]
    assert A.shape == (n, n)
    W = np.array(A, dtype=np.float64, order="F")
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    T = np.zeros(max(n - 1, 1), dtype=np.float64)
    if not want_mag:
        info = _load().oracle_pfonly(n, _dp(W), max(n, 1), _ip(ipiv), _dp(T), nthreads)
        return ipiv[:n], T[:max(n - 1, 0)], int(info)
    M = np.zeros((max(n, 1), max(n, 1)), dtype=np.float64, order="F")
    info = _load().oracle_pfonly_mag(n, _dp(W), max(n, 1), _ip(ipiv), _dp(T), _dp(M), max(n, 1), nthreads)
    Tm = np.array([M[k + 1, k] if k % 2 == 0 else 0.0 for k in range(n - 1)]) if n > 1 else np.zeros(0)
    return ipiv[:n], T[:max(n - 1, 0)], int(info), Tm


def logpf_pfonly(A: np.ndarray, nthreads: int = 1):
    """(log|Pf|, sign, info) by the Pfaffian-only reduction."""
    ipiv, T, info = pfonly(A, nthreads=nthreads)
    if info == ENONFINITE:
        return float("nan"), 0, info
    la, s = logpf_from_factors(A.shape[0], ipiv, T)
    return la, s, info


def pfonly_c128(A: np.ndarray, want_mag: bool = False):
    """Pfaffian-only reduction of the complex skew matrix whose strict lower
    triangle A holds: (ipiv, T, info) with ipiv[k+1] (k even) the interchange of
    step k, the other ipiv[j] = j, T[k] (k even) the pivots and the odd entries
    0; info = n for odd n, ENONFINITE for a non-finite pivot column, else
    1 + the first even k with T[k] = 0, or 0.  Pf(A) = (-1)^{s + n/2} prod T[k].

    want_mag: a fourth item, the magnitude sum of each T[k] (|input| plus
    |l_i v_j| + |v_i l_j| per update that reached it, moved with the entry by
    the interchanges; 0 at the odd entries), as ``ltlt`` gives for real input."""
    n = A.shape[0]
    Lw = np.tril(np.asarray(A, dtype=np.complex128), -1)
    W = Lw - Lw.T
    M = np.abs(W) if want_mag else None
    ipiv = np.arange(n, dtype=np.int32)
    T = np.zeros(max(n - 1, 0), dtype=np.complex128)
    Tm = np.zeros(max(n - 1, 0))

    def out(info):
        return (ipiv, T, info, Tm) if want_mag else (ipiv, T, info)

    if n % 2 == 1:
        return out(n)
    for k in range(0, n - 1, 2):
        col = W[k + 1:, k]
        if not np.all(np.isfinite(col)):
            return out(ENONFINITE)
        key = col.real * col.real + col.imag * col.imag
        p = k + 1 + int(np.argmax(key))
        ipiv[k + 1] = p
        if p != k + 1:
            W[[k + 1, p], :] = W[[p, k + 1], :]
            W[:, [k + 1, p]] = W[:, [p, k + 1]]
            if want_mag:
                M[[k + 1, p], :] = M[[p, k + 1], :]
                M[:, [k + 1, p]] = M[:, [p, k + 1]]
        alpha = W[k + 1, k]
        T[k] = alpha
        if want_mag:
            Tm[k] = M[k + 1, k]
        if k + 2 < n and alpha != 0:
            l = W[k + 2:, k] / alpha
            v = W[k + 2:, k + 1].copy()
            W[k + 2:, k + 2:] += np.outer(l, v) - np.outer(v, l)
            if want_mag:
                al, av = np.abs(l), np.abs(v)
                M[k + 2:, k + 2:] += np.outer(al, av) + np.outer(av, al)
    for k in range(0, n - 1, 2):
        if T[k] == 0:
            return out(k + 1)
    return out(0)


def t_tolerance_c128(T_mag: np.ndarray) -> np.ndarray:
    """Per-entry bound for |T_a[k] - T_b[k]| between two complex Pfaffian-only
    reductions along the same interchanges: a sum of m complex products formed
    with real arithmetic is within sqrt(2) gamma_(m+2) of its magnitude sum
    (Higham, section 3.6); T[k] (k even) collects at most k + 1 terms; twice
    that for the two evaluations."""
    k = np.arange(T_mag.size, dtype=np.float64)
    return 2.0 * np.sqrt(2.0) * gamma(k + 3.0) * T_mag


def logpf_c128_from_factors(n: int, ipiv: np.ndarray, T: np.ndarray):
    """(log|Pf|, phase) with phase = Pf / |Pf| (0 when Pf = 0), in index order."""
    if n == 0:
        return 0.0, 1.0 + 0.0j
    if n % 2 == 1:
        return float("-inf"), 0.0j
    s = int(np.count_nonzero(ipiv[:n] != np.arange(n)))
    ph = -1.0 + 0.0j if (s + n // 2) % 2 else 1.0 + 0.0j
    la = 0.0
    for k in range(0, n - 1, 2):
        t = complex(T[k])
        if t == 0:
            return float("-inf"), 0.0j
        a = abs(t)
        la += math.log(a)
        ph *= t / a
    return la, ph


def cdiv(a, b):
    """a / b for complex128 arrays or scalars by Smith's method with true
    divisions (scaled by the larger component of b): for real operands it is
    the real division exactly."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    ar, ai, br, bi = a.real, a.imag, b.real, b.imag
    big = np.abs(br) >= np.abs(bi)
    with np.errstate(divide="ignore", invalid="ignore"):
        r1 = bi / br
        d1 = br + bi * r1
        r2 = br / bi
        d2 = br * r2 + bi
        re = np.where(big, (ar + ai * r1) / d1, (ar * r2 + ai) / d2)
        im = np.where(big, (ai - ar * r1) / d1, (ai * r2 - ar) / d2)
    return re + 1j * im


def ltlt_c128(A: np.ndarray, want_mag: bool = False):
    """Partially pivoted LTL^T of the complex skew matrix whose strict lower
    triangle A holds: P A P^T = L T L^T, L unit lower triangular with
    L[:, 0] = e_0, T complex skew tridiagonal (T(k+1, k) = T[k], T(k, k+1) = -T[k]).
    Each step k = 0 .. n-2 is the real elimination step with the complex pivot
    key: p = the first index >= k+1 maximising |A[p,k]|^2 = re^2 + im^2 (each
    product rounded); rows and columns k+1 and p interchanged (the multipliers
    already stored in earlier columns move with their rows); T[k] = A[k+1, k];
    l = A[k+2:, k] / T[k] (0 when T[k] = 0); A[k+2:, k+2:] := (A + l v^T) - v l^T
    with v = A[k+2:, k+1]; l is then kept in column k, so that L[i, j] (i > j >= 1)
    is LT[i, j-1], as for real input.  Returns (LT, ipiv, T, info): ipiv[0] = 0,
    ipiv[j] the interchange of step j-1; info ENONFINITE for a non-finite pivot
    column, else 1 + the first even k with T[k] = 0, else 0 (the real rule).

    want_mag: a fifth item M (n x n): M[i, j] (i > j) the sum of the magnitudes
    of the terms entry (i, j) accumulated (|input| plus |l_i v_j| + |v_i l_j| per
    update, moved with the entry by the interchanges), so that M[k+1, k] belongs
    to T[k] and M[i, j-1] to the numerator of L[i, j]."""
    n = A.shape[0]
    Lw = np.tril(np.asarray(A, dtype=np.complex128), -1)
    W = Lw - Lw.T
    M = np.abs(W) if want_mag else None
    ipiv = np.arange(n, dtype=np.int32)
    T = np.zeros(max(n - 1, 0), dtype=np.complex128)
    info = 0
    for k in range(0, n - 1):
        col = W[k + 1:, k]
        if not np.all(np.isfinite(col)):
            info = ENONFINITE
            break
        key = col.real * col.real + col.imag * col.imag
        p = k + 1 + int(np.argmax(key))
        ipiv[k + 1] = p
        if p != k + 1:
            W[[k + 1, p], :] = W[[p, k + 1], :]
            W[:, [k + 1, p]] = W[:, [p, k + 1]]
            if want_mag:
                M[[k + 1, p], :] = M[[p, k + 1], :]
                M[:, [k + 1, p]] = M[:, [p, k + 1]]
        alpha = W[k + 1, k]
        T[k] = alpha
        if k + 2 < n:
            l = cdiv(W[k + 2:, k], alpha) if alpha != 0 else np.zeros(n - k - 2, dtype=np.complex128)
            v = W[k + 2:, k + 1].copy()
            # the strict lower triangle as the definition reads; the upper one is
            # its negative (so an interchange reads exactly what lower storage holds)
            U = np.tril((W[k + 2:, k + 2:] + np.outer(l, v)) - np.outer(v, l), -1)
            W[k + 2:, k + 2:] = U - U.T
            W[k + 2:, k] = l
            if want_mag:
                al, av = np.abs(l), np.abs(v)
                M[k + 2:, k + 2:] += np.outer(al, av) + np.outer(av, al)
    if info == 0:
        for k in range(0, n - 1, 2):
            if T[k] == 0:
                info = k + 1
                break
    LT = np.tril(W, -1)
    return (LT, ipiv, T, info, M) if want_mag else (LT, ipiv, T, info)


def t_tolerance_c128_full(T_mag: np.ndarray) -> np.ndarray:
    """Per-entry bound for |T_a[k] - T_b[k]| between two complex LTL^T
    factorizations along the same interchanges: T[k] collects at most 2k + 1
    complex products (two per earlier step), each sum within sqrt(2) gamma_(m+2)
    of its magnitude sum (Higham, section 3.6); twice that for the two."""
    k = np.arange(T_mag.size, dtype=np.float64)
    return 2.0 * np.sqrt(2.0) * gamma(2.0 * k + 3.0) * T_mag


def l_tolerance_c128(L: np.ndarray, num_mag: np.ndarray, alpha: np.ndarray, alpha_mag: np.ndarray,
                     col: np.ndarray) -> np.ndarray:
    """Per-entry bound for |L_a[i,j] - L_b[i,j]| of the complex factorization:
    L[i,j] = c_i / alpha with c_i and alpha (step j-1) each within the bound of
    ``t_tolerance_c128_full``, plus the rounding of the two complex divisions
    (Smith's method: a few u each)."""
    m = 2.0 * np.asarray(col, dtype=np.float64) + 1.0
    g = 2.0 * np.sqrt(2.0) * gamma(m)
    a = np.abs(alpha)
    return (g * num_mag + np.abs(L) * g * alpha_mag) / a + 16.0 * U_F64 * np.abs(L)


def solve_c128(LT: np.ndarray, ipiv: np.ndarray, T: np.ndarray, B: np.ndarray):
    """X = P^T L^{-T} T^{-1} L^{-1} P B with the complex factors (plain
    transposes: A is complex skew, A^T = -A).  As the real solve: the
    interchanges in order, forward substitution with L (L[i,j] = LT[i,j-1]),
    the tridiagonal T by Gaussian elimination with partial pivoting (row i+1
    taken as pivot row when |T(i+1,i)|^2 > |running diagonal|^2, squares of
    rounded products), back substitution, L^T, the interchanges in reverse.
    Returns (X, info): info = n for odd n, 1 + the first even k with T[k] = 0,
    or the elimination's own zero pivot, else 0."""
    n = LT.shape[0]
    X = np.array(B, dtype=np.complex128)
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    if n == 0:
        return X, 0
    if n % 2 == 1:
        return X, n
    for k in range(0, n - 1, 2):
        if T[k] == 0:
            return X, k + 1
    c2 = lambda z: z.real * z.real + z.imag * z.imag
    for j in range(1, n):
        p = int(ipiv[j])
        if p != j:
            X[[j, p], :] = X[[p, j], :]
    for j in range(1, n):
        X[j + 1:, :] = X[j + 1:, :] - np.outer(LT[j + 1:, j - 1], X[j, :])
    dd = np.zeros(n, dtype=np.complex128)
    du = np.zeros(n, dtype=np.complex128)
    du2 = np.zeros(n, dtype=np.complex128)
    dl = np.zeros(n, dtype=np.complex128)
    dl[:n - 1] = T
    du[:n - 1] = -T
    for i in range(n - 1):
        if c2(dd[i]) >= c2(dl[i]):
            if dd[i] == 0:
                return X, i + 1
            f = complex(cdiv(dl[i], dd[i]))
            dd[i + 1] = dd[i + 1] - f * du[i]
            X[i + 1, :] = X[i + 1, :] - f * X[i, :]
        else:
            f = complex(cdiv(dd[i], dl[i]))
            dd[i] = dl[i]
            t = dd[i + 1]
            dd[i + 1] = du[i] - f * t
            du[i] = t
            if i + 2 < n:
                du2[i] = du[i + 1]
                du[i + 1] = -f * du2[i]
            tb = X[i, :].copy()
            X[i, :] = X[i + 1, :]
            X[i + 1, :] = tb - f * X[i, :]
    if dd[n - 1] == 0:
        return X, n
    X[n - 1, :] = cdiv(X[n - 1, :], dd[n - 1])
    X[n - 2, :] = cdiv(X[n - 2, :] - du[n - 2] * X[n - 1, :], dd[n - 2])
    for i in range(n - 3, -1, -1):
        X[i, :] = cdiv(X[i, :] - du[i] * X[i + 1, :] - du2[i] * X[i + 2, :], dd[i])
    for j in range(n - 1, 0, -1):   # x_j -= L[i, j] x_i, i = j+1 .. n-1 in order
        acc = X[j, :].copy()
        for i in range(j + 1, n):
            acc = acc - LT[i, j - 1] * X[i, :]
        X[j, :] = acc
    for j in range(n - 1, 0, -1):
        p = int(ipiv[j])
        if p != j:
            X[[j, p], :] = X[[p, j], :]
    return X, 0


def pfaffian_bruteforce_complex(A) -> complex:
    """Pfaffian by expansion along the first row, in Python complex arithmetic
    (exact for small Gaussian-integer entries), for n <= 10."""
    M = [[complex(x) for x in row] for row in np.asarray(A)]
    n = len(M)

    def pf(idx):
        m = len(idx)
        if m == 0:
            return 1.0 + 0.0j
        if m % 2 == 1:
            return 0.0j
        i0 = idx[0]
        total = 0.0j
        for t in range(1, m):
            a = M[i0][idx[t]]
            if a == 0:
                continue
            rest = idx[1:t] + idx[t + 1:]
            total += (-1) ** (t + 1) * a * pf(rest)
        return total

    return pf(list(range(n)))


def pf_ratio(A: np.ndarray, U: np.ndarray, V: np.ndarray, nthreads: int = 1):
    """(log|ratio|, sign, info) of Pf(B) / Pf(A), B = A + U V^T - V U^T, from two
    Pfaffians.  Pf(A) = 0 leaves the ratio undefined: (nan, 0, info of A)."""
    A = np.asarray(A, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64).reshape(A.shape[0], -1)
    V = np.asarray(V, dtype=np.float64).reshape(A.shape[0], -1)
    S = full_from_lower(A)
    B = S + (U @ V.T - V @ U.T)
    la_a, s_a, info_a = logpf(S, nthreads=nthreads)
    if s_a == 0:
        n = A.shape[0]
        return float("nan"), 0, (info_a if info_a != 0 else n)
    la_b, s_b, _ = logpf(B, nthreads=nthreads)
    if s_b == 0:
        return float("-inf"), 0, 0
    return la_b - la_a, s_b * s_a, 0


def solve(LT: np.ndarray, ipiv: np.ndarray, T: np.ndarray, B: np.ndarray):
    """X = P^T L^{-T} T^{-1} L^{-1} P B with the oracle's factors; returns (X, info)."""
    n = LT.shape[0]
    X = np.array(B, dtype=np.float64, order="F")
    if X.ndim == 1:
        X = X.reshape(-1, 1, order="F")
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    Tc = np.ascontiguousarray(T, dtype=np.float64)
    if Tc.size == 0:
        Tc = np.zeros(1)
    LTc = np.asfortranarray(LT, dtype=np.float64)
    info = _load().oracle_solve(n, X.shape[1], _dp(LTc), max(n, 1), _ip(ipiv), _dp(Tc), _dp(X), max(n, 1))
    return X, int(info)


# ----------------------------------------------------------------------------
# Definitions written out in Python/numpy
# ----------------------------------------------------------------------------

def pfaffian_bruteforce(A) -> Fraction:
    """Exact Pfaffian by expansion along the first row (n <= 10).

    ``A`` may hold Python ints, Fractions or floats (converted exactly to
    Fractions); the strict upper triangle A[i][j], i < j, is used.
    """
    n = len(A)
    assert n <= 12
    M = [[Fraction(A[i][j]) for j in range(n)] for i in range(n)]

    def pf(idx):
        m = len(idx)
        if m == 0:
            return Fraction(1)
        if m % 2 == 1:
            return Fraction(0)
        i0 = idx[0]
        total = Fraction(0)
        for t in range(1, m):
            a = M[i0][idx[t]]
            if a == 0:
                continue
            rest = idx[1:t] + idx[t + 1:]
            term = a * pf(rest)
            total += term if (t % 2 == 1) else -term
        return total

    return pf(list(range(n)))


def full_from_lower(A: np.ndarray) -> np.ndarray:
    """Skew matrix from the strict lower triangle of A."""
    Lw = np.tril(np.asarray(A, dtype=np.float64), -1)
    return Lw - Lw.T


def reconstruct(LT: np.ndarray, ipiv: np.ndarray, T: np.ndarray):
    """(L, Tm, perm) with P A P^T = L Tm L^T and (P A P^T)[i,j] = A[perm[i], perm[j]]."""
    n = LT.shape[0]
    L = np.eye(n)
    for j in range(1, n):
        L[j + 1:, j] = LT[j + 1:, j - 1]
    Tm = np.zeros((n, n))
    for k in range(n - 1):
        Tm[k + 1, k] = T[k]
        Tm[k, k + 1] = -T[k]
    perm = np.arange(n)
    for j in range(1, n):
        p = int(ipiv[j])
        perm[[j, p]] = perm[[p, j]]
    return L, Tm, perm


def recon_residual(A0: np.ndarray, LT: np.ndarray, ipiv: np.ndarray, T: np.ndarray) -> float:
    """|| P A P^T - L T L^T ||_F / (n ||A||_F) for the skew matrix given by tril(A0, -1)."""
    n = A0.shape[0]
    if n == 0:
        return 0.0
    S = full_from_lower(A0)
    L, Tm, perm = reconstruct(LT, ipiv, T)
    PAP = S[np.ix_(perm, perm)]
    R = PAP - L @ Tm @ L.T
    nrm = np.linalg.norm(S)
    return float(np.linalg.norm(R) / (n * nrm)) if nrm > 0 else float(np.linalg.norm(R))


def skr2k(alpha: float, A: np.ndarray, B: np.ndarray, beta: float, C: np.ndarray) -> np.ndarray:
    """Strict lower triangle of beta C + alpha (A B^T - B A^T); the rest of C is returned unchanged."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    upd = A @ B.T - B @ A.T
    out = np.array(C, dtype=np.float64, order="F")
    low = np.tril(np.ones(out.shape, dtype=bool), -1)
    out[low] = (beta * out + alpha * upd)[low]
    return out


def skr2k_error_bound(alpha: float, A: np.ndarray, B: np.ndarray, beta: float, C: np.ndarray,
                      u: float = 2.0 ** -53) -> np.ndarray:
    """Entrywise bound on |computed - exact| for skr2k in working precision u.

    Any summation order of the 2k products plus the scaling obeys
    |err| <= gamma_{2k+2} (|beta||C| + |alpha| (|A||B|^T + |B||A|^T)),
    gamma_m = m u / (1 - m u).
    """
    k = A.shape[1]
    m = 2 * k + 2
    g = m * u / (1 - m * u)
    aA, aB = np.abs(A), np.abs(B)
    return g * (abs(beta) * np.abs(C) + abs(alpha) * (aA @ aB.T + aB @ aA.T))


def backward_error(A0: np.ndarray, X: np.ndarray, B: np.ndarray) -> float:
    """max_j ||b_j - A x_j||_inf / (||A||_inf ||x_j||_inf + ||b_j||_inf), A skew from tril(A0,-1)."""
    S = full_from_lower(A0)
    R = B - S @ X
    anrm = np.abs(S).sum(axis=1).max() if S.size else 0.0
    num = np.abs(R).max(axis=0)
    den = anrm * np.abs(X).max(axis=0) + np.abs(B).max(axis=0)
    return float((num / den).max()) if num.size else 0.0


def gflops_nominal(n: int, seconds: float) -> float:
    """GFLOP/s on the nominal n^3/3 flop count of the paired factorization."""
    return (n ** 3 / 3.0) / seconds / 1e9


def nominal_flops_steps(n: int, k0: int, k1: int) -> float:
    """Nominal flops of elimination steps k0..k1-1: sum of (n-k-1)^2 (n^3/3 in total)."""
    return float(sum((n - k - 1) ** 2 for k in range(k0, k1)))


def logdet_lu(A_full: np.ndarray):
    """(sign, log|det|) by LAPACK's partially pivoted LU (numpy.linalg.slogdet)."""
    s, ld = np.linalg.slogdet(A_full)
    return float(s), float(ld)


def isclose_log(a: float, b: float) -> float:
    """Relative error used for log|Pf|: |a-b| / max(1, |b|)."""
    if math.isinf(a) and math.isinf(b) and (a > 0) == (b > 0):
        return 0.0
    return abs(a - b) / max(1.0, abs(b))
