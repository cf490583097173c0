"""GPU parity of the low-rank Pfaffian ratio (skf_pf_ratio, through the C ABI)
against the oracle, which divides the Pfaffians of the updated and the original
matrix.  The GPU path uses the Schur-complement identity with one solve through
resident factors instead, so the two agree to a rounding bound derived from the
conditioning (below), and sign for sign.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U_RND = 2.0 ** -53


@pytest.fixture(scope="module")
def skf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_05238_amd import skf as s
    s.lib()
    return s


def _factors(skf, A):
    LT = skf.to_device_colmajor(A)
    ipiv, T, info = skf.ltlt(LT)
    return LT, ipiv, T, info


def _ratio(skf, fac, U, V):
    LT, ipiv, T, _ = fac
    la, sg, info = skf.pf_ratio(LT, ipiv, T, skf.to_device_colmajor(U), skf.to_device_colmajor(V))
    return float(la.item()), int(sg.item()), info


def ratio_tol(S, U, V, la_ref=0.0):
    """Bound on |log|ratio|_GPU - log|ratio|_oracle|, to first order in the backward
    errors, each taken as sqrt(n) u ||.||_2 (the probabilistic bound of Higham and
    Mary, 2019), with a safety factor of 8 for the constants and growth.
    d log|Pf(M)| = tr(M^-1 dM) / 2 for skew M, so
    * the identity (solve with backward error dA): dK = -W^T A^-1 dA X and
      |tr(K^-1 dK)| = |tr(X K^-1 X^T dA)| <= m ||X K^-1 X^T||_2 ||dA||_2
      (W^T A^-1 = -X^T; the middle matrix has rank m = 2r);
    * each of the oracle's two Pfaffians: |tr(M^-1 dM)| <= ||M^-1||_* ||dM||_2;
    plus 64 u max(1, |log|ratio||) for the final logarithms and their sums."""
    n, r = U.shape
    W = np.hstack([U, V])
    X = np.linalg.solve(S, W)
    J = np.block([[np.zeros((r, r)), np.eye(r)], [-np.eye(r), np.zeros((r, r))]])
    K = W.T @ X - J
    B = S + (U @ V.T - V @ U.T)
    _, R = np.linalg.qr(X)
    xkx = np.linalg.norm(R @ np.linalg.inv(K) @ R.T, 2)
    sA = np.linalg.svd(S, compute_uv=False)
    sB = np.linalg.svd(B, compute_uv=False)
    e = math.sqrt(n) * U_RND
    ident = 0.5 * 2 * r * xkx * sA[0] * e
    orc = 0.5 * e * ((1.0 / sA).sum() * sA[0] + (1.0 / sB).sum() * sB[0])
    return 8.0 * (ident + orc) + 64 * U_RND * max(1.0, abs(la_ref))


@pytest.mark.parametrize("n,r", [(2, 1), (64, 1), (64, 32), (300, 2), (300, 5), (1000, 1), (1000, 32),
                                 (2048, 3)])
def test_ratio_parity(skf, oracle_mod, gen, n, r):
    A = gen.skew_gaussian(n, 9500 + n)
    rng = np.random.default_rng(n + r)
    U = rng.standard_normal((n, r))
    V = rng.standard_normal((n, r))
    fac = _factors(skf, A)
    assert fac[3] == 0
    la, sg, info = _ratio(skf, fac, U, V)
    la_r, s_r, info_r = oracle_mod.pf_ratio(A, U, V, nthreads=8)
    tol = ratio_tol(oracle_mod.full_from_lower(A), U, V, la_r)
    print(f"n={n} r={r}: {la!r} vs {la_r!r}, |d| = {abs(la - la_r):.3e}, bound {tol:.3e}")
    assert info == info_r == 0 and sg == s_r
    assert abs(la - la_r) <= tol


def oracle_full(A):
    Lw = np.tril(A, -1)
    return Lw - Lw.T


def test_ratio_closed_form_and_no_change(skf, gen):
    n = 200
    d = np.linspace(0.5, 3.0, n // 2) * np.where(np.arange(n // 2) % 2 == 0, 1.0, -1.0)
    A = np.zeros((n, n))
    for i in range(n // 2):
        A[2 * i + 1, 2 * i], A[2 * i, 2 * i + 1] = d[i], -d[i]
    fac = _factors(skf, A)
    for t in (0.25, 2.0, -1.5):
        U = np.zeros((n, 1))
        V = np.zeros((n, 1))
        U[0, 0], V[1, 0] = t, 1.0
        la, sg, info = _ratio(skf, fac, U, V)
        want = (d[0] - t) / d[0]
        assert info == 0 and sg == np.sign(want) and abs(la - math.log(abs(want))) <= 1e-14
    # U = V: the update is zero, so the ratio is 1 up to rounding
    G = gen.skew_gaussian(300, 4)
    U = np.random.default_rng(5).standard_normal((300, 4))
    la, sg, info = _ratio(skf, _factors(skf, G), U, U)
    assert info == 0 and sg == 1 and abs(la) <= ratio_tol(oracle_full(G), U, U)


def test_ratio_degenerate(skf, gen):
    from paper_2408_05238_amd import skf as s
    A = gen.skew_gaussian(100, 6)
    fac = _factors(skf, A)
    # r = 0: ratio 1
    la, sg, info = s.pf_ratio(fac[0], fac[1], fac[2], s.colmajor(100, 0), s.colmajor(100, 0))
    assert info == 0 and int(sg.item()) == 1 and float(la.item()) == 0.0
    # a rank beyond the supported maximum is an argument error
    with pytest.raises(s.SkfError):
        _ratio(skf, fac, np.ones((100, 33)), np.ones((100, 33)))
    # non-finite update
    U = np.ones((100, 1))
    U[17, 0] = np.nan
    la, sg, info = _ratio(skf, fac, U, np.ones((100, 1)))
    assert info == s.ENONFINITE and sg == 0 and math.isnan(la)
    # updated matrix singular: U = t e_0, V = e_1 with t = d_0 makes block 0 vanish
    # (powers of two, so every step of the solve is exact)
    n = 20
    Bd = np.zeros((n, n))
    for i in range(n // 2):
        Bd[2 * i + 1, 2 * i], Bd[2 * i, 2 * i + 1] = 2.0, -2.0
    U = np.zeros((n, 1))
    V = np.zeros((n, 1))
    U[0, 0], V[1, 0] = 2.0, 1.0
    la, sg, info = _ratio(skf, _factors(skf, Bd), U, V)
    assert info == 0 and ((sg == 0 and la == -math.inf) or la < -30)


def test_ratio_undefined_for_singular_a(skf, gen):
    # odd order: A singular, the ratio undefined; the outcome is the solve's (n)
    A = gen.skew_gaussian(101, 7)
    la, sg, info = _ratio(skf, _factors(skf, A), np.ones((101, 2)), np.arange(202.0).reshape(101, 2))
    assert info == 101 and sg == 0 and math.isnan(la)
    # a zero row and column: a zero pivot
    Z = gen.skew_gaussian(64, 8).copy()
    Z[:, 9] = 0.0
    Z[9, :] = 0.0
    fac = _factors(skf, Z)
    la, sg, info = _ratio(skf, fac, np.ones((64, 1)), np.arange(64.0).reshape(64, 1))
    assert info == fac[3] > 0 and sg == 0 and math.isnan(la)


def test_ratio_n16384_property(skf):
    """At n = 16384 (beyond the oracle's reach) the ratio through the resident
    factors equals the quotient of two Pfaffian-only reductions on the GPU, the
    updated matrix formed explicitly: both sides are parity-tested paths, and
    the log difference of two Pfaffians near e^35000 carries their rounding,
    64 u (|log|Pf(A)|| + |log|Pf(B)||) at most."""
    import torch
    from paper_2408_05238_amd import inputs
    n = 16384
    A = inputs.skew_gaussian(n, 2, inputs.STREAM_A)
    d0 = skf.to_device_colmajor(A)
    del A
    LT = d0.clone()
    ipiv, T, info = skf.ltlt(LT)
    assert info == 0
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    U = torch.randn(1, n, device="cuda", dtype=torch.float64, generator=g).t()
    V = torch.randn(1, n, device="cuda", dtype=torch.float64, generator=g).t()
    la_r, sg_r, info_r = skf.pf_ratio(LT, ipiv, T, U, V)
    del LT
    Bm = d0.clone()
    Bm.add_(U @ V.t() - V @ U.t())
    la_b, sg_b, _ = skf.logpf(Bm)
    del Bm
    la_a, sg_a, _ = skf.logpf(d0)
    la_r, la_b, la_a = float(la_r.item()), float(la_b.item()), float(la_a.item())
    print(f"log|ratio| {la_r!r} vs {la_b - la_a!r}")
    assert info_r == 0 and int(sg_r.item()) == int(sg_b.item()) * int(sg_a.item())
    assert abs(la_r - (la_b - la_a)) <= 64 * U_RND * (abs(la_a) + abs(la_b))
