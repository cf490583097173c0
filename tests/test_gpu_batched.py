"""GPU parity of the batched persistent factorization and of the batched
Pfaffian-only reduction against the CPU oracle, and batch-composition
independence (a matrix's result is the same alone and in any mix, bit for bit)."""
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
    la, sg, info = skf.logpf_batched(mats)
    la, sg, info = _host(la), _host(sg), _host(info)
    la_r, s_r, _ = oracle_mod.logpf(mats_h[0])
    assert sg[0] == s_r and oracle_mod.isclose_log(la[0], la_r) <= 1e-12
    assert info[1] == skf.ENONFINITE
    assert sg[2] == 0 and la[2] == -np.inf
    # the full factorization reports it too, for a NaN and for an infinity
    for bad in (np.nan, np.inf):
        mats_h[1][50, 3] = bad
        mats = [skf.to_device_colmajor(A) for A in mats_h]
        _, _, info_f, _, _ = skf.ltlt_batched(mats)
        info_f = _host(info_f)
        assert info_f[1] == skf.ENONFINITE and info_f[0] == 0, (bad, info_f)


SOLVE_NS = [0, 1, 2, 3, 4, 6, 64, 65, 66, 100, 130, 257, 300, 511, 512]
SOLVE_NRHS = [1, 2, 3, 1, 0, 4, 1, 2, 5, 1, 3, 1, 2, 1, 3]


def test_solve_batched(skf, oracle_mod, gen):
    """One launch over uneven orders and right-hand-side counts: every solution
    has backward error <= 1e-13 with its matrix and matches the oracle's solve
    with the same factors; odd orders report n, and the result of a matrix is
    the same bits alone as in the mix."""
    import torch
    ns, nrs = SOLVE_NS, SOLVE_NRHS
    mats_h = [gen.batch_matrix(n, 17, b) for b, n in enumerate(ns)]
    mats = [skf.to_device_colmajor(A) for A in mats_h]
    _, _, _, ipivs, Ts = skf.ltlt_batched(mats)
    Bs_h = [gen.gaussian(n, r, 100 + b) for b, (n, r) in enumerate(zip(ns, nrs))]
    Bs = [skf.to_device_colmajor(B) for B in Bs_h]
    info = _host(skf.solve_batched(mats, ipivs, Ts, Bs)).tolist()
    assert info == [n if n % 2 else 0 for n in ns]
    for b, n in enumerate(ns):
        if n % 2 or n == 0 or nrs[b] == 0:
            continue
        X = _host(Bs[b])
        assert oracle_mod.backward_error(mats_h[b], X, Bs_h[b]) <= 1e-13, (n, b)
        Xr, inf2 = oracle_mod.solve(_host(mats[b]), _host(ipivs[b]), _host(Ts[b]), Bs_h[b])
        assert inf2 == 0
        assert np.abs(X - Xr).max() <= 1e-9 * np.abs(Xr).max() * max(1.0, n / 64), (n, b)
    # alone vs in the mix: bitwise
    b = ns.index(300)
    B1 = skf.to_device_colmajor(Bs_h[b])
    assert _host(skf.solve_batched([mats[b]], [ipivs[b]], [Ts[b]], [B1])).tolist() == [0]
    assert np.array_equal(_host(B1), _host(Bs[b]))
    torch.cuda.synchronize()


def test_solve_batched_wide_orders_and_singular(skf, oracle_mod, gen):
    """Orders above the batched factorization's reach, factored one by one: 700
    (sixteen rows per lane) stays in the one launch, 1100 takes the single-matrix
    solve; a zero first row and column gives info 1."""
    ns = [700, 1100, 40]
    mats_h = [gen.skew_gaussian(n, 300 + n) for n in ns]
    mats_h[2][:, 0] = 0.0
    mats_h[2][0, :] = 0.0
    mats, ipivs, Ts = [], [], []
    for A in mats_h:
        dA = skf.to_device_colmajor(A)
        ip, T, _ = skf.ltlt(dA)
        mats.append(dA)
        ipivs.append(ip)
        Ts.append(T)
    Bs_h = [gen.gaussian(n, 2, 700 + n) for n in ns]
    Bs = [skf.to_device_colmajor(B) for B in Bs_h]
    info = _host(skf.solve_batched(mats, ipivs, Ts, Bs)).tolist()
    assert info == [0, 0, 1]
    for b in range(2):
        X = _host(Bs[b])
        assert oracle_mod.backward_error(mats_h[b], X, Bs_h[b]) <= 1e-13, ns[b]
        Xr, _ = oracle_mod.solve(_host(mats[b]), _host(ipivs[b]), _host(Ts[b]), Bs_h[b])
        assert np.abs(X - Xr).max() <= 1e-9 * np.abs(Xr).max() * max(1.0, ns[b] / 64), ns[b]


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
    # the Pfaffian-only path: the same bits on every run, the same Pfaffian as the factorization
    pf = []
    for _ in range(2):
        la2, sg2, info2, ip2, _ = skf.pfonly_batched([skf.to_device_colmajor(A) for A in mats_h])
        pf.append((_host(la2), _host(sg2), _host(info2), [_host(t) for t in ip2]))
    assert all(np.array_equal(x, y) for x, y in zip(pf[0][:3], pf[1][:3]))
    assert all(np.array_equal(x, y) for x, y in zip(pf[0][3], pf[1][3]))
    assert np.array_equal(pf[0][1], a[1])
    assert np.abs(pf[0][0] - a[0]).max() <= 1e-12 * np.abs(a[0]).max()


@pytest.mark.parametrize("seed", [7, 23])
def test_pfonly_batched_parity(skf, oracle_mod, gen, seed):
    """The Pfaffian-only reduction against the oracle's: interchanges equal,
    pivots and log|Pf| within rounding, signs and outcomes equal."""
    mats_h = [gen.batch_matrix(n, seed, b) for b, n in enumerate(SIZES)]
    mats = [skf.to_device_colmajor(A) if A.shape[0] > 0 else skf.colmajor(0, 0) for A in mats_h]
    la, sg, info, ipivs, Ts = skf.pfonly_batched(mats)
    la, sg, info = _host(la), _host(sg), _host(info)
    for b, (A, n) in enumerate(zip(mats_h, SIZES)):
        ip_r, T_r, info_r = oracle_mod.pfonly(A) if n > 0 else (np.zeros(0, np.int32), np.zeros(0), 0)
        la_r, s_r = oracle_mod.logpf_from_factors(n, ip_r, T_r) if n > 0 else (0.0, 1)
        assert info[b] == info_r, (b, n, info[b], info_r)
        assert sg[b] == s_r, (b, n)
        if n % 2 == 1:
            assert la[b] == -np.inf
            continue
        assert oracle_mod.isclose_log(la[b], la_r) <= 1e-12, (b, n, la[b], la_r)
        if n >= 2:
            ip, T = _host(ipivs[b]), _host(Ts[b])
            assert np.array_equal(ip, ip_r), (b, n)
            assert np.all(T[1::2] == 0.0)
            assert np.abs(T[0::2] - T_r[0::2]).max() <= 1e-11 * np.abs(T_r[0::2]).max(), (b, n)


def test_pfonly_batched_alone_equals_mixed_and_edges(skf, oracle_mod, gen):
    mats_h = [gen.batch_matrix(n, 29, b) for b, n in enumerate([300, 64, 512, 130, 2, 256, 18])]
    # an exactly singular matrix (a zero row/column) and a block-diagonal one with a known Pfaffian
    Z = gen.batch_matrix(40, 29, 99).copy()
    Z[:, 5] = 0.0
    Z[5, :] = 0.0
    d = np.linspace(0.5, 2.0, 20) * np.where(np.arange(20) % 3 == 0, -1.0, 1.0)
    J = np.zeros((40, 40))
    for i in range(20):
        J[2 * i, 2 * i + 1], J[2 * i + 1, 2 * i] = d[i], -d[i]
    mats_h += [Z, J]
    mixed = [skf.to_device_colmajor(A) for A in mats_h]
    la_m, sg_m, info_m, ip_m, _ = skf.pfonly_batched(mixed)
    la_m, sg_m, info_m = _host(la_m), _host(sg_m), _host(info_m)
    for b, A in enumerate(mats_h):
        la_1, sg_1, info_1, ip_1, _ = skf.pfonly_batched([skf.to_device_colmajor(A)])
        assert _host(la_1)[0] == la_m[b] and _host(sg_1)[0] == sg_m[b] and _host(info_1)[0] == info_m[b]
        assert np.array_equal(_host(ip_1[0]), _host(ip_m[b]))
    assert sg_m[-2] == 0 and la_m[-2] == -np.inf and info_m[-2] > 0
    assert sg_m[-1] == int(np.sign(np.prod(d))) and abs(la_m[-1] - np.log(np.abs(d)).sum()) <= 1e-13 * 40


def test_batched_uses_only_the_strict_lower_triangle(skf, gen):
    """Both batched kernels give the same bits when the diagonal and the strict
    upper triangle hold NaN, and leave those places unwritten."""
    sizes = [2, 3, 34, 130, 300, 512]
    clean = [gen.batch_matrix(n, 31, b) for b, n in enumerate(sizes)]
    dirty = []
    for A in clean:
        D = A.copy()
        D[np.triu_indices(A.shape[0])] = np.nan
        dirty.append(D)
    for run in (skf.pfonly_batched, skf.ltlt_batched):
        mc = [skf.to_device_colmajor(A) for A in clean]
        md = [skf.to_device_colmajor(A) for A in dirty]
        rc, rd = run(mc), run(md)
        for k in range(3):  # log|Pf|, sign, outcome
            assert np.array_equal(_host(rc[k]), _host(rd[k]), equal_nan=True), (run.__name__, k)
        for b, n in enumerate(sizes):
            assert np.array_equal(_host(rc[3][b]), _host(rd[3][b])), (run.__name__, n)
            assert np.array_equal(_host(rc[4][b]), _host(rd[4][b])), (run.__name__, n)
            got = _host(md[b])
            assert np.all(np.isnan(got[np.triu_indices(n)])), (run.__name__, n)
            assert np.array_equal(np.tril(_host(mc[b]), -1), np.tril(got, -1)), (run.__name__, n)
