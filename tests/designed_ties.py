"""Skew matrices with a known factorization, exact ties in the pivot columns and
exactly representable arithmetic (a test-input construction, no part of either
computation).

A = P^T (L0 T0 L0^T) P with
  * L0 unit lower triangular with L0[:,0] = e_0 and entries in
    {0, +-1/4, +-1/2, +-3/4, +-1} below the diagonal: every entry of magnitude 1
    in column k+1 makes |A^(k)[i,k]| equal to the pivot |T0[k]|, an exact tie;
  * T0 skew tridiagonal with T0[k] in {+-1/2, +-1, +-2} (powers of two, so every
    multiplier c / T0[k] is exact, by division or by reciprocal);
  * P a product of interchanges j <-> p_j at a random subset of steps, applied in
    order; the entries of L0 that would otherwise out-rank or tie with the pivot
    row ahead of p_j in the pre-interchange column are halved, so that partial
    pivoting with ties to the lowest index chooses exactly p_j.
Every value the elimination forms is a multiple of 2^-6 below 2^24 in
magnitude, so any order of evaluation, with or without fused multiply-adds, is
exact: a correct factorization returns ipiv = the designed interchanges,
T = T0 and L = L0 bit for bit.
"""
from __future__ import annotations

import numpy as np


def designed(n: int, seed: int, p_one: float = 0.05, p_swap: float = 0.1):
    """(A, ipiv, T0, L0): A full skew (column-major friendly float64), the
    interchanges, the tridiagonal's subdiagonal and L0 (n x n)."""
    rng = np.random.default_rng(seed)
    vals = np.array([0.25, 0.5, 0.75])
    L0 = np.eye(n)
    for j in range(1, n - 1):
        m = n - j - 1
        x = rng.choice(vals, size=m) * rng.choice([-1.0, 1.0], size=m)
        x[rng.random(m) < 0.4] = 0.0
        ones = rng.random(m) < p_one
        x[ones] = rng.choice([-1.0, 1.0], size=int(ones.sum()))
        L0[j + 1:, j] = x
    T0 = rng.choice([0.5, 1.0, 2.0], size=max(n - 1, 0)) * rng.choice([-1.0, 1.0], size=max(n - 1, 0))
    ipiv = np.arange(n, dtype=np.int32)
    for j in range(1, n - 1):
        if rng.random() < p_swap:
            ipiv[j] = rng.integers(j + 1, n)
    # Pre-interchange column k (step k, r = k+1): the row now at index i ends at
    # f(i) after the interchanges r, r+1, ... are applied, and holds
    # T0[k] * L0[f(i), r] (L0[r, r] = 1 is the pivot).  Rows k+1 .. p-1 must stay
    # strictly below magnitude 1.
    F = np.arange(n)                        # F_r[i]: final position of the row at i (interchanges r.. applied)
    for r in range(n - 1, 0, -1):
        p = int(ipiv[r])
        F[[r, p]] = F[[p, r]]
        if p == r:
            continue
        f = F[r:p]
        col = L0[f, r]
        hit = (f != r) & (np.abs(col) == 1.0)
        L0[f[hit], r] *= 0.5
    # B = L0 T L0^T (exact: integer multiples of 2^-5 well inside 2^53), A = P^T B P
    Tm = np.zeros((n, n))
    for k in range(n - 1):
        Tm[k + 1, k], Tm[k, k + 1] = T0[k], -T0[k]
    B = (L0 @ Tm) @ L0.T
    perm = np.arange(n)
    for j in range(1, n):                   # (P B P^T)[i, j] = B[perm[i], perm[j]] after the interchanges
        q = int(ipiv[j])
        perm[[j, q]] = perm[[q, j]]
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    A = B[np.ix_(inv, inv)]
    A = np.tril(A, -1) - np.tril(A, -1).T
    return np.asfortranarray(A), ipiv, T0, L0


def tie_steps(A_oracle_gap) -> int:
    """Number of steps whose two largest candidates tie exactly (gap 0)."""
    return int(np.count_nonzero(np.asarray(A_oracle_gap) == 0.0))
