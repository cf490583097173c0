"""Exact ties between pivot candidates in different workgroups.

The matrices of tests/designed_ties.py have a known factorization, exact ties
(candidates of equal magnitude spread over the whole column) at nearly every
step, designed interchanges, and exactly representable arithmetic.  The GPU
must choose the lowest index on every tie, as the oracle does: ipiv, T and L
equal the design (and the oracle) bit for bit, in both panel widths.
"""
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


CASES = [(300, 11, "128"), (1000, 12, "128"), (4096, 13, "128"), (1000, 14, "64"), (4500, 15, "64"),
         (2000, 16, None), (1000, 17, "32"), (2000, 18, "16"), (4096, 19, "256")]


@pytest.mark.parametrize("n,seed,nb", CASES, ids=[f"n{c[0]}-nb{c[2] or 'auto'}" for c in CASES])
def test_ties_across_workgroups(skf, oracle_mod, n, seed, nb, monkeypatch):
    from designed_ties import designed
    if nb:
        monkeypatch.setenv("SKF_NB", nb)
    A, ipiv, T0, L0 = designed(n, seed)
    ref = oracle_mod.ltlt(A, nthreads=8)
    assert np.array_equal(ref.ipiv, ipiv) and np.array_equal(ref.T, T0)
    assert np.count_nonzero(ref.gap == 0.0) > n // 2
    dA = skf.to_device_colmajor(A)
    ip, T, info = skf.ltlt(dA)
    ip, T = ip.cpu().numpy(), T.cpu().numpy()
    LT = dA.cpu().numpy()
    assert info == 0
    bad = np.nonzero(ip != ipiv)[0]
    assert bad.size == 0, (bad[:5], ip[bad[:5]], ipiv[bad[:5]])
    assert np.array_equal(T[:n - 1], T0)
    assert np.array_equal(np.tril(LT, -2), np.tril(ref.LT, -2))
