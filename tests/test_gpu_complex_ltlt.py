"""GPU parity of the complex (complex128) LTL^T and of the solve with its
factors (skf_ltlt_c128, skf_solve_c128, through the C ABI) against the oracle's
numpy factorization and solve: interchanges bit for bit, T and every L entry
within the summation-error bound of its magnitude sum, the subdiagonal of the
output equal to T, log|Pf| and the phase against the oracle; real input gives
the real factorization's interchanges; the solve against the oracle's solve
with the same (GPU) factors and by its backward error with A.  Every panel
width (64 and, with SKF_NB=32 or 16, 32 or 16 steps per panel) is covered; at
n = 4096 and 16384 (no stored oracle result) the checks are properties: log|Pf|
against the Pfaffian-only reduction (a different elimination order) and the
solve's backward error; at n = 33000 (the width-16 panel's range, 516
workgroups) real input against the real factorization's interchanges and the
solve's backward error on complex input."""
from __future__ import annotations

import math

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


@pytest.fixture(params=["nb64", "nb32", "nb16"])
def width(request, monkeypatch):
    monkeypatch.delenv("SKF_NB", raising=False)
    if request.param != "nb64":
        monkeypatch.setenv("SKF_NB", request.param[2:])
    return request.param


def _cgauss(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return np.tril(X, -1) - np.tril(X, -1).T


def _factor(skf, A):
    dA = skf.to_device_colmajor(np.asarray(A, dtype=np.complex128))
    ipiv, T, info = skf.ltlt_c128(dA)
    return dA, ipiv, T, info


def _check_factors(oracle_mod, A, LT, ip, T, info):
    n = A.shape[0]
    LT_r, ip_r, T_r, info_r, M = oracle_mod.ltlt_c128(A, want_mag=True)
    assert info == info_r
    assert np.array_equal(ip, ip_r), int(np.argmax(ip != ip_r))
    if n < 2:
        return
    Tm = np.array([M[k + 1, k] for k in range(n - 1)])
    tol = oracle_mod.t_tolerance_c128_full(Tm)
    d = np.abs(T - T_r)
    assert np.all(d <= tol), (int(np.argmax(d - tol)), d.max())
    # the subdiagonal of the output holds T
    assert np.array_equal(np.array([LT[k + 1, k] for k in range(n - 1)]), T)
    for c in range(n - 2):
        Lg, Lr = LT[c + 2:, c], LT_r[c + 2:, c]
        tl = oracle_mod.l_tolerance_c128(Lr, M[c + 2:, c], T_r[c], Tm[c], c + 1)
        dl = np.abs(Lg - Lr)
        assert np.all(dl <= tl), (c, int(np.argmax(dl - tl)), dl.max())
    la, ph = oracle_mod.logpf_c128_from_factors(n, ip, T)
    la_r, ph_r = oracle_mod.logpf_c128_from_factors(n, ip_r, T_r)
    if la_r != -math.inf:
        assert abs(la - la_r) <= 1e-12 * max(1.0, abs(la_r))
        assert abs(ph - ph_r) <= float(np.sum(tol[0::2] / np.abs(T_r[0::2]))) + 4 * n * 2.0 ** -53


@pytest.mark.parametrize("n", [1, 2, 3, 4, 64, 65, 130, 512, 1024])
def test_complex_ltlt_parity(skf, oracle_mod, width, n):
    A = _cgauss(n, 8100 + n)
    dA, ipiv, T, info = _factor(skf, A)
    print(f"complex ltlt n={n} {width}", flush=True)
    _check_factors(oracle_mod, A, dA.cpu().numpy(), ipiv.cpu().numpy(), T.cpu().numpy(), info)


def test_complex_ltlt_real_input_and_edges(skf, oracle_mod, gen):
    from paper_2408_05238_amd import skf as s
    R = gen.skew_gaussian(300, 12)
    dA, ipiv, T, info = _factor(skf, R.astype(np.complex128))
    dR = skf.to_device_colmajor(R)
    ipr, Tr, infor = skf.ltlt(dR)
    assert info == infor == 0 and np.array_equal(ipiv.cpu().numpy(), ipr.cpu().numpy())
    assert not np.any(T.cpu().numpy().imag)
    # a zero row and column: info 1 + the first even zero pivot, as the oracle
    Z = _cgauss(100, 2)
    Z[:, 17] = 0
    Z[17, :] = 0
    dZ, ipz, Tz, infz = _factor(skf, Z)
    _check_factors(oracle_mod, Z, dZ.cpu().numpy(), ipz.cpu().numpy(), Tz.cpu().numpy(), infz)
    N = _cgauss(100, 4)
    N[60, 10] = complex(np.nan, 1.0)
    assert _factor(skf, N)[3] == s.ENONFINITE
    E = s.colmajor(0, 0, dtype=__import__("torch").complex128)
    ip0, T0, inf0 = s.ltlt_c128(E)
    assert inf0 == 0 and ip0.numel() == 0


@pytest.mark.parametrize("n,nrhs", [(2, 1), (64, 3), (130, 5), (512, 2), (1000, 4)])
def test_complex_solve_parity(skf, oracle_mod, width, n, nrhs):
    A = _cgauss(n, 8300 + n)
    rng = np.random.default_rng(n)
    B = rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs))
    dA, ipiv, T, info = _factor(skf, A)
    assert info == 0
    dB = skf.to_device_colmajor(B)
    assert skf.solve_c128(dA, ipiv, T, dB) == 0
    X = dB.cpu().numpy()
    Xr, inf2 = oracle_mod.solve_c128(dA.cpu().numpy(), ipiv.cpu().numpy(), T.cpu().numpy(), B)
    assert inf2 == 0
    assert np.abs(X - Xr).max() <= 1e-9 * np.abs(Xr).max() * max(1.0, n / 64)
    r = np.abs(A @ X - B).max(axis=0)
    eta = r / (np.abs(A).sum(1).max() * np.abs(X).max(axis=0) + np.abs(B).max(axis=0))
    assert eta.max() <= 1e-13, eta


def test_complex_solve_singular_and_odd(skf):
    A = _cgauss(7, 3)
    dA, ipiv, T, _ = _factor(skf, A)
    dB = skf.to_device_colmajor(np.ones((7, 2), dtype=np.complex128))
    assert skf.solve_c128(dA, ipiv, T, dB) == 7
    Z = _cgauss(20, 4)
    Z[:, 0] = 0
    Z[0, :] = 0
    dZ, ipz, Tz, infz = _factor(skf, Z)
    assert infz == 1
    B = np.arange(40, dtype=np.float64).reshape(20, 2) + 1j
    dB = skf.to_device_colmajor(B)
    assert skf.solve_c128(dZ, ipz, Tz, dB) == 1
    assert np.array_equal(dB.cpu().numpy(), B)   # left as it is


@pytest.mark.parametrize("n,nb", [(4096, None), (16384, None), (16384, "32")])
def test_complex_ltlt_full_size_properties(skf, n, nb, monkeypatch):
    """Orders of the complex workload: log|Pf| and the phase from the factors
    against the Pfaffian-only reduction of the same matrix (1e-12 relative), and
    the solve's backward error with A (two right-hand sides)."""
    import torch
    from paper_2408_05238_amd import inputs
    monkeypatch.delenv("SKF_NB", raising=False)
    if nb:
        monkeypatch.setenv("SKF_NB", nb)
    A = inputs.skew_gaussian_c128(n, 2)
    dA0 = skf.to_device_colmajor(A)
    dA = dA0.clone()
    print(f"complex ltlt full size n={n} nb={nb}", flush=True)
    ipiv, T, info = skf.ltlt_c128(dA)
    assert info == 0
    la, ph = skf.logpf_c128_from_factors(n, ipiv, T)
    ip2, T2, info2 = skf.pfonly_c128(dA0)
    la2, ph2 = skf.logpf_c128_from_factors(n, ip2, T2)
    la, la2 = float(la.item()), float(la2.item())
    ph, ph2 = complex(ph.item()), complex(ph2.item())
    assert info2 == 0 and abs(la - la2) <= 1e-12 * abs(la2) and abs(ph - ph2) <= 1e-8, (la, la2, ph, ph2)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    dB = skf.to_device_colmajor(B)
    assert skf.solve_c128(dA, ipiv, T, dB) == 0
    # residual with A = S - S^T (S the strict lower triangle of the input)
    S = torch.tril(dA0, -1)
    Xd = dB
    R = (S @ Xd - S.T @ Xd) - skf.to_device_colmajor(B)
    anorm = float((S.abs().sum(1) + S.abs().sum(0)).max())
    eta = (R.abs().amax(0) / (anorm * Xd.abs().amax(0) + torch.from_numpy(np.abs(B).max(0)).to(Xd.device))).max()
    assert float(eta) <= 1e-13, float(eta)


def test_complex_ltlt_width16_range(skf, monkeypatch):
    """n = 33000: beyond the 32-step panel's reach (516 panel workgroups, four
    per CU with 16 steps per panel).  A real matrix as complex input gives the
    real factorization's interchanges (T real, equal to the real T within the
    two evaluations' rounding); complex input gives a solve with backward error
    at most 1e-13."""
    import torch
    from paper_2408_05238_amd import inputs
    monkeypatch.delenv("SKF_NB", raising=False)
    n = 33000
    assert skf.lib().skf_ltlt_c128_workspace(n) > 0
    R = skf.to_device_colmajor(inputs.skew_gaussian(n, 3, inputs.STREAM_A))
    C = R.to(torch.complex128)
    print(f"complex ltlt n={n} real input", flush=True)
    ipc, Tc, infc = skf.ltlt_c128(C)
    del C
    ipr, Tr, infr = skf.ltlt(R)
    del R
    assert infc == infr == 0
    assert torch.equal(ipc, ipr)
    assert float(Tc.imag.abs().max()) == 0.0
    assert float(((Tc.real - Tr).abs() / Tr.abs().clamp_min(1e-300)).max()) <= 1e-9
    del ipc, Tc, ipr, Tr
    torch.cuda.empty_cache()
    print(f"complex ltlt n={n} complex input", flush=True)
    g = torch.Generator(device="cuda").manual_seed(11)
    X = torch.randn(n, n, dtype=torch.complex128, device="cuda", generator=g)
    S = torch.tril(X, -1)
    del X
    A = S.t().contiguous().t()   # column-major; only the strict lower triangle is read
    ipiv, T, info = skf.ltlt_c128(A)
    assert info == 0
    B = torch.randn(n, 2, dtype=torch.complex128, device="cuda", generator=g)
    Bc = B.t().contiguous().t()
    Xs = Bc.clone().t().contiguous().t()
    assert skf.solve_c128(A, ipiv, T, Xs) == 0
    del A
    R2 = (S @ Xs - S.t() @ Xs) - Bc
    anorm = float((S.abs().sum(1) + S.abs().sum(0)).max())
    eta = (R2.abs().amax(0) / (anorm * Xs.abs().amax(0) + Bc.abs().amax(0))).max()
    print(f"complex ltlt n={n}: solve backward error {float(eta):.2e}", flush=True)
    assert float(eta) <= 1e-13
