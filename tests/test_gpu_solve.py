"""GPU parity of the solve and the iterative refinement against the CPU oracle."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def skf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_05238_amd import skf as s
    s.lib()
    return s


def _host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n,nrhs", [(2, 1), (4, 3), (64, 16), (66, 5), (130, 17), (300, 16), (513 - 1, 33)])
def test_solve_parity(skf, oracle_mod, gen, n, nrhs):
    A = gen.skew_gaussian(n, 900 + n)
    B = gen.gaussian(n, nrhs, 901 + n)
    dA = skf.to_device_colmajor(A)
    ipiv, T, info = skf.ltlt(dA)
    assert info == 0
    dB = skf.to_device_colmajor(B)
    info = skf.solve(dA, ipiv, T, dB)
    assert info == 0
    X = _host(dB)
    # backward error of the GPU solution with the original matrix
    assert oracle_mod.backward_error(A, X, B) <= 1e-13
    # against the oracle's solve with the oracle's factors (same pivots)
    f = oracle_mod.ltlt(A)
    Xr, inf2 = oracle_mod.solve(f.LT, f.ipiv, f.T, B)
    assert inf2 == 0
    scale = np.abs(Xr).max()
    assert np.abs(X - Xr).max() <= 1e-9 * scale * max(1.0, n / 64)


def test_solve_odd_singular(skf, gen):
    A = gen.skew_gaussian(7, 3)
    dA = skf.to_device_colmajor(A)
    ipiv, T, _ = skf.ltlt(dA)
    dB = skf.to_device_colmajor(np.ones((7, 2)))
    assert skf.solve(dA, ipiv, T, dB) == 7


def test_solve_zero_pivot_info(skf, gen):
    n = 20
    A = gen.skew_gaussian(n, 4)
    A[:, 0] = 0.0
    A[0, :] = 0.0
    dA = skf.to_device_colmajor(A)
    ipiv, T, info = skf.ltlt(dA)
    assert info == 1
    dB = skf.to_device_colmajor(np.ones((n, 1)))
    assert skf.solve(dA, ipiv, T, dB) == 1


@pytest.mark.parametrize("n", [256, 1000])
def test_refine_fp64_and_fp32(skf, oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 77 + n)
    B = gen.gaussian(n, 16, 78 + n)
    A0 = skf.to_device_colmajor(A)
    dB = skf.to_device_colmajor(B)
    for prec in (skf.PREC_F64, skf.PREC_F32_TRAILING):
        dA = A0.clone() if False else skf.to_device_colmajor(A)
        ipiv, T, info = skf.ltlt(dA, prec=prec)
        assert info == 0
        X, st, iters, berr = skf.solve_refine(A0, dA, ipiv, T, dB, tol=1e-13, maxit=20)
        assert st == 0, (prec, iters, berr)
        assert berr <= 1e-13
        Xh = _host(X)
        assert oracle_mod.backward_error(A, Xh, B) <= 2e-13


@pytest.mark.parametrize("kappa", [1e4, 1e6])
def test_refine_fp32_ill_conditioned(skf, oracle_mod, gen, kappa):
    """A = Q D Q^T with skew 2x2 blocks d_i log-spaced over [1/kappa, 1] and Q
    orthogonal: FP32-trailing factors are too inexact for plain refinement to
    contract on such a matrix, and the GMRES-based correction has to take over."""
    n = 600
    G = gen.gaussian(n, n, 910)
    Q, _ = np.linalg.qr(G)
    d = np.logspace(0.0, -np.log10(kappa), n // 2)
    D = np.zeros((n, n))
    for i, v in enumerate(d):
        D[2 * i, 2 * i + 1], D[2 * i + 1, 2 * i] = v, -v
    A = Q @ D @ Q.T
    A = 0.5 * (A - A.T)
    B = gen.gaussian(n, 16, 911)
    A0 = skf.to_device_colmajor(A)
    dA = skf.to_device_colmajor(A)
    ipiv, T, info = skf.ltlt(dA, prec=skf.PREC_F32_TRAILING)
    assert info == 0
    X, st, iters, berr = skf.solve_refine(A0, dA, ipiv, T, skf.to_device_colmajor(B), tol=1e-13, maxit=10)
    assert st == 0 and berr <= 1e-13, (st, iters, berr)
    assert oracle_mod.backward_error(A, _host(X), B) <= 2e-13


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mixed_precision_workload_n16384(skf, oracle_mod, prec):
    """The mixed-precision workload at its stated size: the n = 16384 skew
    Gaussian matrix of seed 5 with 16 Gaussian right-hand sides of seed 6,
    factored with FP64 or FP32-trailing updates, refined to FP64 backward
    error <= 1e-13; eta recomputed on the host by the oracle's definition."""
    import torch
    from paper_2408_05238_amd import inputs
    n, nrhs = 16384, 16
    print(f"mixed n={n} prec={prec}", flush=True)
    A = inputs.skew_gaussian(n, 5, inputs.STREAM_A)
    B = inputs.gaussian(n, nrhs, 6, inputs.STREAM_B)
    A0 = skf.to_device_colmajor(A)
    dA = A0.clone()
    dB = skf.to_device_colmajor(B)
    p = skf.PREC_F64 if prec == "f64" else skf.PREC_F32_TRAILING
    ipiv, T, info = skf.ltlt(dA, prec=p)
    assert info == 0
    X, st, iters, berr = skf.solve_refine(A0, dA, ipiv, T, dB, tol=1e-13, maxit=20)
    torch.cuda.synchronize()
    print(f"mixed n={n} prec={prec}: status {st}, corrections {iters}, eta {berr:.3e}")
    assert st == 0 and berr <= 1e-13
    del dA, A0
    assert oracle_mod.backward_error(A, _host(X), B) <= 1e-13
