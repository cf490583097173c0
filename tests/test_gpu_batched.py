"""GPU parity of the batched persistent factorization against the CPU oracle,
and batch-composition independence (a matrix's result is the same alone and in
any mix, bit for bit)."""
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


SIZES = [0, 1, 2, 3, 4, 31, 32, 33, 64, 65, 100, 128, 129, 200, 255, 256, 300, 511, 512, 7, 2, 512, 48]


def test_batched_parity(skf, oracle_mod, gen):
    mats_h = [gen.batch_matrix(n, 7, b) for b, n in enumerate(SIZES)]
    mats = [skf.to_device_colmajor(A) if A.shape[0] > 0 else skf.colmajor(0, 0) for A in mats_h]
    la, sg, info, ipivs, Ts = skf.ltlt_batched(mats)
    la, sg, info = _host(la), _host(sg), _host(info)
    for b, (A, n) in enumerate(zip(mats_h, SIZES)):
        ref = oracle_mod.ltlt(A) if n > 0 else None
        la_r, s_r = oracle_mod.logpf_from_factors(n, ref.ipiv, ref.T) if n > 0 else (0.0, 1)
        assert sg[b] == s_r, (b, n)
        assert oracle_mod.isclose_log(la[b], la_r) <= 1e-12, (b, n, la[b], la_r)
        if n >= 2:
            assert info[b] == ref.info
            ip, T = _host(ipivs[b]), _host(Ts[b])
            assert np.array_equal(ip, ref.ipiv), (b, n)
            LT = np.asfortranarray(_host(mats[b]))
            assert oracle_mod.recon_residual(A, LT, ip, T) <= 1e-13
            assert np.abs(T - ref.T).max() <= 1e-11 * np.abs(ref.T).max()


def test_batched_alone_equals_mixed(skf, gen):
    mats_h = [gen.batch_matrix(n, 11, b) for b, n in enumerate([300, 64, 512, 130, 2, 256])]
    mixed = [skf.to_device_colmajor(A) for A in mats_h]
    la_m, sg_m, _, ip_m, T_m = skf.ltlt_batched(mixed)
    for b, A in enumerate(mats_h):
        one = [skf.to_device_colmajor(A)]
        la_1, sg_1, _, ip_1, T_1 = skf.ltlt_batched(one)
        assert _host(la_1)[0] == _host(la_m)[b] and _host(sg_1)[0] == _host(sg_m)[b]
        assert np.array_equal(_host(T_1[0]), _host(T_m[b]))
        assert np.array_equal(_host(one[0]), _host(mixed[b]))


def test_batched_logpf_only_and_nonfinite(skf, oracle_mod, gen):
    mats_h = [gen.batch_matrix(n, 13, b) for b, n in enumerate([40, 90, 41])]
    mats_h[1] = mats_h[1].copy()
    mats_h[1][50, 3] = np.nan
    mats = [skf.to_device_colmajor(A) for A in mats_h]
    la, sg, info, _, _ = skf.ltlt_batched(mats, with_factors=False)
    la, sg, info = _host(la), _host(sg), _host(info)
    la_r, s_r, _ = oracle_mod.logpf(mats_h[0])
    assert sg[0] == s_r and oracle_mod.isclose_log(la[0], la_r) <= 1e-12
    assert info[1] == skf.ENONFINITE
    assert sg[2] == 0 and la[2] == -np.inf


def test_solve_batched(skf, oracle_mod, gen):
    ns = [64, 100, 2]
    mats_h = [gen.batch_matrix(n, 17, b) for b, n in enumerate(ns)]
    mats = [skf.to_device_colmajor(A) for A in mats_h]
    _, _, _, ipivs, Ts = skf.ltlt_batched(mats)
    Bs_h = [gen.gaussian(n, 3, 100 + b) for b, n in enumerate(ns)]
    Bs = [skf.to_device_colmajor(B) for B in Bs_h]
    info = skf.solve_batched(mats, ipivs, Ts, Bs)
    assert _host(info).tolist() == [0, 0, 0]
    for b in range(3):
        assert oracle_mod.backward_error(mats_h[b], _host(Bs[b]), Bs_h[b]) <= 1e-13


def test_batched_repeatable_large_mix(skf, gen):
    """Two launches over the same 300-matrix mix give the same bits (a race
    between the threads of a workgroup would show here)."""
    ns = gen.even_sizes(300, 32, 512, 99).tolist()
    mats_h = [gen.batch_matrix(n, 99, b) for b, n in enumerate(ns)]
    outs = []
    for _ in range(2):
        mats = [skf.to_device_colmajor(A) for A in mats_h]
        la, sg, info, ipivs, Ts = skf.ltlt_batched(mats)
        outs.append((_host(la), _host(sg), _host(info), [_host(t) for t in Ts], [_host(m) for m in mats]))
    a, b = outs
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert all(np.array_equal(x, y) for x, y in zip(a[3], b[3]))
    assert all(np.array_equal(x, y) for x, y in zip(a[4], b[4]))
    la2, sg2, _, _, _ = skf.ltlt_batched([skf.to_device_colmajor(A) for A in mats_h], with_factors=False)
    assert np.array_equal(_host(la2), a[0]) and np.array_equal(_host(sg2), a[1])
