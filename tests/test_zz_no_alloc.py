"""skf_solve_noalloc (fixed device scratch, no workspace argument) against
skf_solve (caller workspace) through the C ABI: the same kernels on the same
inputs, so X must agree bit for bit; two calls in a row, the second smaller, so
the second runs on scratch the first left behind."""
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


def _case(skf, n, nrhs, seed, async_info):
    import torch
    from paper_2408_05238_amd import inputs
    print(f"no-alloc solve case n={n} nrhs={nrhs} seed={seed} async={async_info}", flush=True)
    A = inputs.skew_gaussian(n, seed, inputs.STREAM_A)
    dA = skf.to_device_colmajor(A)
    ipiv, T, info = skf.ltlt(dA)
    assert info == 0
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, nrhs))
    X1 = skf.to_device_colmajor(B)
    X2 = skf.to_device_colmajor(B)
    assert skf.solve(dA, ipiv, T, X1) == 0
    if async_info:
        d = torch.full((1,), -7, dtype=torch.int32, device=dA.device)
        skf.solve_noalloc(dA, ipiv, T, X2, dinfo=d)
        torch.cuda.synchronize()
        assert int(d.item()) == 0
    else:
        assert skf.solve_noalloc(dA, ipiv, T, X2) == 0
    x1, x2 = X1.cpu().numpy(), X2.cpu().numpy()
    assert np.array_equal(x1, x2), float(np.abs(x1 - x2).max())
    import oracle
    assert oracle.backward_error(A, x2, B) <= 1e-13


def test_solve_noalloc_matches_solve_twice(skf):
    _case(skf, 4096, 16, 31, False)   # largest accepted order, one full pass of right-hand sides
    _case(skf, 602, 5, 32, True)      # smaller order on the scratch the first call left behind


def test_solve_noalloc_limits(skf):
    import torch
    dA = skf.colmajor(4098, 4098).zero_()
    ip = torch.zeros(4098, dtype=torch.int32, device="cuda")
    T = torch.zeros(4097, dtype=torch.float64, device="cuda")
    B = skf.colmajor(4098, 1).zero_()
    with pytest.raises(skf.SkfError) as e:
        skf.solve_noalloc(dA, ip, T, B)
    assert e.value.code == skf.ESCRATCH
    # odd order: singular, info = n, as skf_solve
    n = 5
    from paper_2408_05238_amd import inputs
    A = inputs.skew_gaussian(n, 3, inputs.STREAM_A)
    dA = skf.to_device_colmajor(A)
    ipiv, T, _ = skf.ltlt(dA)
    B = skf.colmajor(n, 2).fill_(1.0)
    assert skf.solve_noalloc(dA, ipiv, T, B) == n
