"""GPU parity of the blocked Pfaffian-only reduction (skf_pfonly, and skf_logpf /
skf_pfaffian, which are built on it) against the oracle's Pfaffian-only
reduction: interchanges bit for bit, the odd entries of ipiv and T exactly the
identity and zero, the even pivots within a rounding tolerance, log|Pf|, sign
and outcome.  At n = 16384 the Pfaffian is checked against the stored oracle
results of the full factorization (the same Pfaffian by a different reduction).
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LOGPF_TOL = 1e-12   # |d log|Pf|| / max(1, |log|Pf||)




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


def _pf_gpu(skf, A, prec=0):
    dA = skf.to_device_colmajor(A)
    ipiv, T, info = skf.pfonly(dA, prec=prec)
    return _host(ipiv), _host(T), info


def _check_against_oracle(oracle_mod, A, ip, T, info):
    n = A.shape[0]
    ip_r, T_r, info_r, Tm = oracle_mod.pfonly(A, nthreads=8, want_mag=True)
    assert info == info_r, (n, info, info_r)
    assert np.array_equal(ip, ip_r), (n, int(np.argmax(ip != ip_r)))
    assert np.all(T[1::2] == 0.0) and np.all(ip[0::2] == np.arange(0, n, 2))
    if n >= 2:
        # each even pivot within the summation-error bound of its magnitude sum
        d = np.abs(T - T_r)
        tol = oracle_mod.t_tolerance(Tm, full=False)
        assert np.all(d <= tol), (n, int(np.argmax(d - tol)), d.max())
    la, s = oracle_mod.logpf_from_factors(n, ip, T)
    la_r, s_r = oracle_mod.logpf_from_factors(n, ip_r, T_r)
    assert s == s_r and oracle_mod.isclose_log(la, la_r) <= LOGPF_TOL, (n, la, la_r)


@pytest.mark.parametrize("n", [2, 4, 6, 64, 66, 128, 130, 256, 258, 600, 1000, 2048, 4096])
def test_pfonly_parity(skf, oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 9100 + n)
    ip, T, info = _pf_gpu(skf, A)
    _check_against_oracle(oracle_mod, A, ip, T, info)


@pytest.mark.parametrize("n,nb", [(300, "64"), (778, "64"), (2048, "64"), (4500, "64"), (300, "128"),
                                  (2048, "128"), (4096, "128"), (300, "32"), (2048, "32"), (778, "16"),
                                  (2048, "16"), (300, "256"), (2048, "256"), (6000, "256")])
def test_pfonly_parity_nb(skf, oracle_mod, gen, n, nb, monkeypatch):
    """Each panel width forced, whatever the tuning table picks for n."""
    monkeypatch.setenv("SKF_NB", nb)
    A = gen.skew_gaussian(n, 9300 + n)
    ip, T, info = _pf_gpu(skf, A)
    _check_against_oracle(oracle_mod, A, ip, T, info)


@pytest.mark.parametrize("n", [1, 3, 129])
def test_pfonly_odd(skf, gen, n):
    ip, T, info = _pf_gpu(skf, gen.skew_gaussian(n, 5))
    assert info == n
    assert np.array_equal(ip, np.arange(n)) and np.all(T == 0.0)
    la, sg, _ = skf.logpf(skf.to_device_colmajor(gen.skew_gaussian(n, 5)))
    assert int(sg.item()) == 0 and float(la.item()) == -math.inf


def test_pfonly_empty(skf):
    from paper_2408_05238_amd import skf as s
    A = s.colmajor(0, 0)
    ip, T, info = s.pfonly(A)
    assert info == 0 and ip.numel() == 0 and T.numel() == 0


@pytest.mark.parametrize("where", [(7, 0), (150, 90)])
def test_pfonly_nonfinite(skf, oracle_mod, gen, where):
    A = gen.skew_gaussian(200, 5)
    A[where] = np.nan
    _, _, info = _pf_gpu(skf, A)
    assert info == skf.ENONFINITE == oracle_mod.pfonly(A)[2]


def test_pfonly_singular_and_known(skf, oracle_mod, gen):
    # a zero row/column: Pf = 0, the outcome names the first zero pivot as the oracle does
    Z = gen.skew_gaussian(300, 8).copy()
    Z[:, 123] = 0.0
    Z[123, :] = 0.0
    ip, T, info = _pf_gpu(skf, Z)
    _check_against_oracle(oracle_mod, Z, ip, T, info)
    assert info > 0
    # block diagonal with 2x2 blocks [[0, -d], [d, 0]] (lower entry d): Pf = (-1)^{n/2} prod d
    n = 260
    d = np.linspace(0.5, 2.0, n // 2) * np.where(np.arange(n // 2) % 3 == 0, -1.0, 1.0)
    J = np.zeros((n, n))
    for i in range(n // 2):
        J[2 * i + 1, 2 * i], J[2 * i, 2 * i + 1] = d[i], -d[i]
    ip, T, info = _pf_gpu(skf, J)
    la, s = oracle_mod.logpf_from_factors(n, ip, T)
    assert info == 0
    assert s == int(np.sign(np.prod(d))) * (-1) ** (n // 2)
    assert abs(la - np.log(np.abs(d)).sum()) <= 1e-13 * n


def test_pfonly_repeatable_and_logpf_route(skf, oracle_mod, gen):
    """Two runs give the same bits, and skf_logpf gives exactly the Pfaffian of
    skf_pfonly's factors (it runs the same reduction)."""
    A = gen.skew_gaussian(1030, 41)
    r1 = _pf_gpu(skf, A)
    r2 = _pf_gpu(skf, A)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1]) and r1[2] == r2[2] == 0
    la, sg, info = skf.logpf(skf.to_device_colmajor(A))
    ipiv, T, _ = skf.pfonly(skf.to_device_colmajor(A))
    la_f, s_f = skf.logpf_from_factors(1030, ipiv, T)
    assert info == 0 and int(sg.item()) == int(s_f.item()) and float(la.item()) == float(la_f.item())
    la_h, s_h = oracle_mod.logpf_from_factors(1030, r1[0], r1[1])
    assert s_h == int(s_f.item()) and oracle_mod.isclose_log(float(la_f.item()), la_h) <= 1e-14


def test_pfonly_f32_trailing(skf, oracle_mod, gen):
    n = 512
    A = gen.skew_gaussian(n, 123)
    ip, T, info = _pf_gpu(skf, A, prec=skf.PREC_F32_TRAILING)
    assert info == 0
    la_g, s_g = oracle_mod.logpf_from_factors(n, ip, T)
    la_r, s_r, _ = oracle_mod.logpf_pfonly(A, nthreads=8)
    assert s_g == s_r and oracle_mod.isclose_log(la_g, la_r) <= 1e-5


@pytest.mark.parametrize("seed", [2, 3, 4])
def test_pfonly_n16384_against_stored_oracle(skf, seed):
    import torch
    from paper_2408_05238_amd import inputs
    N = 16384
    path = os.path.join(HERE, "golden", f"ltlt_n{N}_s{seed}.npz")
    assert os.path.exists(path), path
    g = np.load(path)
    A = inputs.skew_gaussian(N, seed, inputs.STREAM_A)
    dA = skf.to_device_colmajor(A)
    del A
    la, sg, info = skf.logpf(dA)
    torch.cuda.synchronize()
    la, sg = float(la.item()), int(sg.item())
    print(f"seed {seed}: log|Pf| {la!r} vs {float(g['logabs'])!r}")
    assert info == 0 and sg == int(g["sign"])
    assert abs(la - float(g["logabs"])) <= LOGPF_TOL * max(1.0, abs(float(g["logabs"])))


@pytest.mark.parametrize("nb", [None, "256"])
def test_pfonly_n16384_against_stored_pfonly_oracle(skf, nb, monkeypatch):
    """The launch configuration of skf_logpf at n = 16384 (panel_pf_kernel with
    256 workgroups), and the same with the widest panel (nb = 256, one
    workgroup per CU): interchanges bit for bit against the oracle's
    Pfaffian-only mode (tests/golden/pfonly_n16384_s2.npz), every even pivot
    within its per-entry bound, log|Pf| and sign."""
    import torch
    from paper_2408_05238_amd import inputs
    import oracle
    if nb:
        monkeypatch.setenv("SKF_NB", nb)
    print(f"pfonly n=16384 nb={nb or 'auto'}", flush=True)
    N = 16384
    g = np.load(os.path.join(HERE, "golden", f"pfonly_n{N}_s2.npz"))
    A = inputs.skew_gaussian(N, 2, inputs.STREAM_A)
    dA = skf.to_device_colmajor(A)
    del A
    ipiv, T, info = skf.pfonly(dA)
    torch.cuda.synchronize()
    ip, Th = _host(ipiv), _host(T)[:N - 1]
    assert info == int(g["info"]) == 0
    assert np.array_equal(ip, g["ipiv"]), int(np.argmax(ip != g["ipiv"]))
    d = np.abs(Th - g["T"])
    tol = oracle.t_tolerance(g["T_mag"], full=False)
    k = int(np.argmax(d / np.maximum(tol, 1e-300)))
    print(f"pfonly n={N}: max |dT| / bound = {d[k] / tol[k]:.3e} at k = {k}")
    assert np.all(d <= tol)
    la, sg = oracle.logpf_from_factors(N, ip, Th)
    assert sg == int(g["sign"]) and oracle.isclose_log(la, float(g["logabs"])) <= LOGPF_TOL
