"""GPU parity of the complex (complex128) Pfaffian-only reduction
(skf_pfonly_c128, through the C ABI) against the oracle's numpy reduction:
interchanges bit for bit, the odd entries exactly the identity / zero, each
pivot within the complex summation-error bound of its magnitude sum, log|Pf|
and the phase.  Both forms are covered: the blocked one (panel kernel plus the
real matrix-core trailing update on the real and imaginary planes; both panel
widths) and the unblocked one (SKF_C128_UNBLOCKED=1); at n = 2048 and 4096 the
reference is the oracle's stored result (tests/golden/pfonly_c128_n*_s2.npz,
written by tests/golden/make_golden.py).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U_RND = 2.0 ** -53


PATHS = ["blocked", "unblocked", "blocked-nb64"]


@pytest.fixture(params=PATHS)
def path(request, monkeypatch):
    monkeypatch.delenv("SKF_C128_UNBLOCKED", raising=False)
    monkeypatch.delenv("SKF_NB", raising=False)
    if request.param == "unblocked":
        monkeypatch.setenv("SKF_C128_UNBLOCKED", "1")
    elif request.param == "blocked-nb64":
        monkeypatch.setenv("SKF_NB", "64")
    return request.param


@pytest.fixture(scope="module")
def skf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_05238_amd import skf as s
    s.lib()
    return s


def _cgauss(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return np.tril(X, -1) - np.tril(X, -1).T


def _run(skf, A):
    dA = skf.to_device_colmajor(np.asarray(A, dtype=np.complex128))
    before = np.ascontiguousarray(dA.cpu().numpy()).view(np.uint64)
    ipiv, T, info = skf.pfonly_c128(dA)
    la, ph = skf.logpf_c128_from_factors(A.shape[0], ipiv, T)
    after = np.ascontiguousarray(dA.cpu().numpy()).view(np.uint64)
    assert np.array_equal(before, after), "the input must not be modified"
    return ipiv.cpu().numpy(), T.cpu().numpy(), info, float(la.item()), complex(ph.item())


def _check(oracle_mod, n, ip, T, info, la, ph, ip_r, T_r, info_r, Tm):
    assert info == info_r == 0
    assert np.array_equal(ip, ip_r), int(np.argmax(ip != ip_r))
    assert np.all(T[1::2] == 0) and np.all(ip[0::2] == np.arange(0, n, 2))
    d = np.abs(T - T_r)
    tol = oracle_mod.t_tolerance_c128(Tm)
    assert np.all(d <= tol), (int(np.argmax(d - tol)), d.max())
    la_r, ph_r = oracle_mod.logpf_c128_from_factors(n, ip_r, T_r)
    assert abs(la - la_r) <= 1e-12 * max(1.0, abs(la_r))
    # each pivot's relative difference turns the phase by at most that much, and
    # the product of n/2 unit factors rounds at most 4u per factor
    ph_tol = float(np.sum(tol[0::2] / np.abs(T_r[0::2]))) + 4 * n * U_RND
    assert abs(ph - ph_r) <= ph_tol, (ph, ph_r, ph_tol)


@pytest.mark.parametrize("n", [2, 4, 6, 64, 130, 512, 1024])
def test_complex_parity(skf, oracle_mod, path, n):
    A = _cgauss(n, 7000 + n)
    ip, T, info, la, ph = _run(skf, A)
    ip_r, T_r, info_r, Tm = oracle_mod.pfonly_c128(A, want_mag=True)
    _check(oracle_mod, n, ip, T, info, la, ph, ip_r, T_r, info_r, Tm)


@pytest.mark.parametrize("n", [2048, 4096])
def test_complex_against_stored_oracle(skf, oracle_mod, n, monkeypatch):
    """The blocked reduction at n = 2048 (32 panel workgroups) and 4096 (64) on the
    complex skew Gaussian matrix of seed 2 (the bench workload at 4096)."""
    import os
    from paper_2408_05238_amd import inputs
    monkeypatch.delenv("SKF_C128_UNBLOCKED", raising=False)
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", f"pfonly_c128_n{n}_s2.npz"))
    print(f"complex golden case n={n}", flush=True)
    ip, T, info, la, ph = _run(skf, inputs.skew_gaussian_c128(n, 2))
    _check(oracle_mod, n, ip, T, info, la, ph, g["ipiv"], g["T"], int(g["info"]), g["T_mag"])


def test_complex_known_values(skf, oracle_mod, path):
    # block diagonal: Pf = prod over blocks of A[2i, 2i+1] = prod(-d_i)
    m = 40
    rng = np.random.default_rng(3)
    d = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    A = np.zeros((2 * m, 2 * m), dtype=np.complex128)
    for i in range(m):
        A[2 * i + 1, 2 * i], A[2 * i, 2 * i + 1] = d[i], -d[i]
    _, _, info, la, ph = _run(skf, A)
    want = np.prod(-d)
    assert info == 0 and abs(math.exp(la) * ph - want) <= 1e-12 * abs(want)
    # a real matrix: the same interchanges as the real Pfaffian-only reduction
    R = _cgauss(200, 5).real
    ip, T, info, _, _ = _run(skf, R)
    ip_r, T_r, _ = skf.pfonly(skf.to_device_colmajor(R))
    assert info == 0 and np.array_equal(ip, ip_r.cpu().numpy())
    assert np.all(T.imag == 0)


def test_complex_edges(skf, oracle_mod, path):
    from paper_2408_05238_amd import skf as s
    ip, T, info, la, ph = _run(skf, _cgauss(9, 1))
    assert info == 9 and np.array_equal(ip, np.arange(9)) and np.all(T == 0) and la == -math.inf and ph == 0
    E = s.colmajor(0, 0, dtype=__import__("torch").complex128)
    ipiv, T0, info = s.pfonly_c128(E)
    assert info == 0 and ipiv.numel() == 0
    Z = _cgauss(100, 2)
    Z[:, 17] = 0
    Z[17, :] = 0
    _, _, info, la, ph = _run(skf, Z)
    assert info == oracle_mod.pfonly_c128(Z)[2] > 0 and ph == 0 and la == -math.inf
    N = _cgauss(100, 4)
    N[60, 10] = complex(np.nan, 1.0)
    _, _, info, _, _ = _run(skf, N)
    assert info == s.ENONFINITE == oracle_mod.pfonly_c128(N)[2]
