"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Pivots are compared bit for bit; T, log|Pf| and the factors within the stated
tolerances; the reconstruction residual ||PAP^T - LTL^T||_F / (n ||A||_F) is
computed on the host from the GPU's own outputs.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

RECON_TOL = 1e-13          # ||PAP^T - LTL^T||_F / (n ||A||_F), FP64
LOGPF_TOL = 1e-12          # |d log|Pf|| / max(1, |log|Pf||)


@pytest.fixture(scope="module")
def skf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_05238_amd import skf as s
    s.lib()
    return s


def _dev(skf, a):
    return skf.to_device_colmajor(a)


def _host(t):
    return t.detach().cpu().numpy()


def _factor_gpu(skf, A, prec=0):
    dA = _dev(skf, A)
    ipiv, T, info = skf.ltlt(dA, prec=prec)
    return np.asfortranarray(_host(dA)), _host(ipiv), _host(T), info


def check_T_L(oracle_mod, ref, LT, T):
    """T and L against the oracle entry by entry, each within the summation-error
    bound of its magnitude sum (oracle.t_tolerance / oracle.l_tolerance)."""
    n = ref.LT.shape[0]
    if n < 2:
        return
    tm = ref.T_mag()
    dT = np.abs(T[:n - 1] - ref.T)
    tolT = oracle_mod.t_tolerance(tm)
    assert np.all(dT <= tolT), (int(np.argmax(dT - tolT)), dT.max())
    if n < 3:
        return
    i, j = np.nonzero(np.tril(np.ones((n, n), bool), -2))   # L[i, j+1] stored at (i, j)
    Lr = ref.LT[i, j]
    tolL = oracle_mod.l_tolerance(Lr, ref.M[i, j], ref.T[j], tm[j], j + 1)
    dL = np.abs(LT[i, j] - Lr)
    assert np.all(dL <= tolL), (int(np.argmax(dL - tolL)), dL.max())


# ---------------------------------------------------------------------------
# skr2k
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,k", [(1, 3), (2, 1), (17, 5), (128, 64), (129, 7), (300, 64), (513, 130), (64, 0)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 1.0), (-0.5, 2.0), (1.5, 0.0)])
def test_skr2k_f64(skf, oracle_mod, n, k, alpha, beta):
    rng = np.random.default_rng(n * 1000 + k)
    A = rng.standard_normal((n, k))
    B = rng.standard_normal((n, k))
    C = rng.standard_normal((n, n))
    if beta == 0.0:
        C[np.tril_indices(n, -1)] = np.nan   # must not be read
    dC = _dev(skf, C)
    skf.skr2k(alpha, _dev(skf, A), _dev(skf, B), beta, dC)
    got = _host(dC)
    Cin = np.nan_to_num(C) if beta == 0.0 else C
    ref = oracle_mod.skr2k(alpha, A, B, beta, Cin)
    bound = oracle_mod.skr2k_error_bound(alpha, A, B, beta, Cin)
    low = np.tril(np.ones((n, n), bool), -1)
    assert np.all(np.abs(got - ref)[low] <= bound[low] + 1e-300)
    assert np.array_equal(got[~low], C[~low], equal_nan=True)   # diagonal/upper untouched


@pytest.mark.parametrize("n,k", [(17, 5), (300, 64), (513, 130)])
def test_skr2k_f32(skf, oracle_mod, n, k):
    rng = np.random.default_rng(7 + n)
    A = rng.standard_normal((n, k))
    B = rng.standard_normal((n, k))
    C = rng.standard_normal((n, n))
    dC = _dev(skf, C)
    skf.skr2k(1.0, _dev(skf, A), _dev(skf, B), 1.0, dC, f32=True)
    got = _host(dC)
    ref = oracle_mod.skr2k(1.0, A, B, 1.0, C)
    # inputs rounded to FP32 (relative 2^-24 each) and FP32 accumulation over 2k terms
    bound = oracle_mod.skr2k_error_bound(1.0, A, B, 0.0, 0 * C, u=2.0 ** -24) * 1.5 + \
        oracle_mod.skr2k_error_bound(0.0, A, B, 1.0, C) + 1e-300
    low = np.tril(np.ones((n, n), bool), -1)
    assert np.all(np.abs(got - ref)[low] <= bound[low])


# ---------------------------------------------------------------------------
# LTL^T parity
# ---------------------------------------------------------------------------
SIZES = [2, 3, 4, 5, 7, 8, 33, 63, 64, 65, 127, 128, 129, 130, 131, 255, 256, 257, 258, 300, 511, 512, 1500]


@pytest.mark.parametrize("n", SIZES)
def test_ltlt_parity(skf, oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 5000 + n)
    ref = oracle_mod.ltlt(A, want_mag=True, nthreads=8)
    assert ref.info == 0
    LT, ipiv, T, info = _factor_gpu(skf, A)
    assert info == 0
    if ref.gap is not None and ref.gap.size:
        assert ref.gap.min() > 1e-10, "seed has a near-tie pivot; pick another"
    assert np.array_equal(ipiv, ref.ipiv), np.nonzero(ipiv != ref.ipiv)[0][:10]
    check_T_L(oracle_mod, ref, LT, T)
    assert oracle_mod.recon_residual(A, LT, ipiv, T) <= RECON_TOL
    # diagonal and strict upper triangle are never written
    assert np.array_equal(np.triu(LT), np.triu(A))
    la_g, s_g = oracle_mod.logpf_from_factors(n, ipiv, T)
    la_r, s_r = oracle_mod.logpf_from_factors(n, ref.ipiv, ref.T)
    assert s_g == s_r and oracle_mod.isclose_log(la_g, la_r) <= LOGPF_TOL


def test_ltlt_worked_4x4(skf, oracle_mod):
    A = np.zeros((4, 4))
    for (i, j), v in {(0, 1): 1, (0, 2): 2, (0, 3): 3, (1, 2): 4, (1, 3): 5, (2, 3): 6}.items():
        A[i, j], A[j, i] = v, -v
    LT, ipiv, T, info = _factor_gpu(skf, A)
    assert info == 0 and ipiv.tolist() == [0, 3, 2, 3]
    np.testing.assert_allclose(T, [-3.0, 6.0, 8.0 / 3.0], rtol=1e-15)
    np.testing.assert_allclose([LT[2, 0], LT[3, 0], LT[3, 1]], [2 / 3, 1 / 3, 5 / 6], rtol=1e-15)


@pytest.mark.parametrize("n", [0, 1])
def test_ltlt_degenerate_sizes(skf, n):
    import torch
    dA = skf.colmajor(n, n)
    ipiv, T, info = skf.ltlt(dA)
    assert info == 0
    if n == 1:
        assert ipiv.cpu().tolist() == [0]


def test_ltlt_lda_larger(skf, oracle_mod, gen):
    n, lda = 200, 257
    A = gen.skew_gaussian(n, 42)
    dA = skf.colmajor(n, n, ld=lda)
    import torch
    dA.copy_(torch.from_numpy(np.asfortranarray(A)))
    ipiv, T, info = skf.ltlt(dA)
    ref = oracle_mod.ltlt(A)
    assert info == 0 and np.array_equal(_host(ipiv), ref.ipiv)
    assert oracle_mod.recon_residual(A, np.asfortranarray(_host(dA)), _host(ipiv), _host(T)) <= RECON_TOL


def test_ltlt_only_lower_read(skf, oracle_mod, gen):
    n = 150
    A = gen.skew_gaussian(n, 9)
    B = A.copy()
    B[np.triu_indices(n)] = np.nan
    LTa, ipa, Ta, _ = _factor_gpu(skf, A)
    LTb, ipb, Tb, info = _factor_gpu(skf, B)
    assert info == 0 and np.array_equal(ipa, ipb) and np.array_equal(Ta, Tb)
    assert np.array_equal(np.tril(LTa, -1), np.tril(LTb, -1))


def test_ltlt_zero_column_info(skf, oracle_mod, gen):
    n = 96
    A = gen.skew_gaussian(n, 3)
    A[:, 0] = 0.0
    A[0, :] = 0.0
    LT, ipiv, T, info = _factor_gpu(skf, A)
    ref = oracle_mod.ltlt(A)
    assert info == ref.info == 1
    assert T[0] == 0.0 and np.array_equal(ipiv, ref.ipiv)


@pytest.mark.parametrize("where", [(7, 0), (150, 90)])
def test_ltlt_nonfinite(skf, oracle_mod, gen, where):
    n = 200
    A = gen.skew_gaussian(n, 5)
    A[where] = np.nan
    _, _, _, info = _factor_gpu(skf, A)
    assert info == skf.ENONFINITE == oracle_mod.ltlt(A).info


@pytest.mark.parametrize("n", [64, 257, 512])
def test_logpf_and_pfaffian_api(skf, oracle_mod, gen, n):
    A = gen.skew_gaussian(n, 77 + n)
    la_r, s_r, _ = oracle_mod.logpf(A)
    la, sg, info = skf.logpf(_dev(skf, A))
    # skf_logpf runs the Pfaffian-only reduction: odd n reports info = n (Pf = 0) as its oracle mode does
    assert info == (n if n % 2 else 0) == oracle_mod.pfonly(A)[2] and int(sg.item()) == s_r
    if n % 2:
        assert s_r == 0 and float(la.item()) == la_r == -math.inf
    else:
        assert oracle_mod.isclose_log(float(la.item()), la_r) <= LOGPF_TOL
    small = A[:10, :10] * 0.5
    pf, info = skf.pfaffian(_dev(skf, small))
    exact = float(oracle_mod.pfaffian_bruteforce(small))
    assert info == 0 and abs(float(pf.item()) - exact) <= 1e-12 * abs(exact)


@pytest.mark.parametrize("n", [3, 5, 101])
def test_logpf_odd(skf, gen, n):
    la, sg, info = skf.logpf(_dev(skf, gen.skew_gaussian(n, 1)))
    assert int(sg.item()) == 0 and float(la.item()) == -math.inf


def test_ltlt_f32_trailing_accuracy(skf, oracle_mod, gen):
    n = 512
    A = gen.skew_gaussian(n, 123)
    LT, ipiv, T, info = _factor_gpu(skf, A, prec=skf.PREC_F32_TRAILING)
    assert info == 0
    r = oracle_mod.recon_residual(A, LT, ipiv, T)
    assert r <= 1e-8, r           # FP32 trailing products: ~u32-level backward error
    ref = oracle_mod.ltlt(A)
    la_g, s_g = oracle_mod.logpf_from_factors(n, ipiv, T)
    la_r, s_r = oracle_mod.logpf_from_factors(n, ref.ipiv, ref.T)
    assert oracle_mod.isclose_log(la_g, la_r) <= 1e-5


def test_ltlt_repeatable(skf, gen):
    A = gen.skew_gaussian(300, 31)
    r1 = _factor_gpu(skf, A)
    r2 = _factor_gpu(skf, A)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[2], r2[2])


@pytest.mark.parametrize("n,nb", [(300, "64"), (777, "64"), (2048, "64"), (4500, "64"), (300, "128"),
                                  (2048, "128"), (4096, "128"), (300, "32"), (1000, "32"), (2048, "32"),
                                  (777, "16"), (2048, "16"), (300, "256"), (777, "256"), (4096, "256"),
                                  (6000, "256")])
def test_ltlt_parity_nb(skf, oracle_mod, gen, n, nb, monkeypatch):
    """Each panel width forced, whatever the tuning table picks for n (the narrow
    panel is also the only one that fits beyond one CU's worth of slots per CU)."""
    monkeypatch.setenv("SKF_NB", nb)
    A = gen.skew_gaussian(n, 6000 + n)
    ref = oracle_mod.ltlt(A, want_mag=True, nthreads=8)
    LT, ipiv, T, info = _factor_gpu(skf, A)
    assert info == 0 and np.array_equal(ipiv, ref.ipiv)
    check_T_L(oracle_mod, ref, LT, T)
    assert oracle_mod.recon_residual(A, LT, ipiv, T) <= RECON_TOL
    la_g, s_g = oracle_mod.logpf_from_factors(n, ipiv, T)
    la_r, s_r = oracle_mod.logpf_from_factors(n, ref.ipiv, ref.T)
    assert s_g == s_r and oracle_mod.isclose_log(la_g, la_r) <= LOGPF_TOL
