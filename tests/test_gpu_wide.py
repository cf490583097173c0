"""Orders beyond the wide panels' reach (n > 32769 on 256 CUs): the planner takes
the narrower panel widths, whose workgroups fit several to a CU.  n = 50000 runs
782 panel workgroups of width 32 (some CUs hold four), n = 98304 runs 1536 of
them (six per CU, the records read in two blocks per step), and n = 40000 the
width-16 panel.  No stored
oracle result exists at these orders (the oracle would take hours), so the
checks are properties that hold at any size: the reconstruction residual
||P A P^T - L T L^T||_F / (n ||A||_F) estimated with Gaussian probes, the
interchange and multiplier invariants (ipiv[j] >= j, |L| <= 1), and log|Pf| and
its sign from the factors against the Pfaffian-only reduction of the same
matrix, a different elimination order (1e-12 relative).  Narrow widths at
small orders are compared with the oracle in test_gpu_ltlt.py,
test_gpu_pfonly.py and test_gpu_ties.py."""
from __future__ import annotations

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

RECON_TOL = 1e-13
LOGPF_TOL = 1e-12


@pytest.fixture(scope="module")
def skf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_05238_amd import skf as s
    s.lib()
    return s


def _apply_P(x, ipiv, transpose=False):
    x = x.copy()
    js = range(len(ipiv) - 1, 0, -1) if transpose else range(1, len(ipiv))
    for j in js:
        p = int(ipiv[j])
        if p != j:
            x[[j, p]] = x[[p, j]]
    return x


BLK = 2048  # columns per block: the checks never form an n x n temporary


def _blocks(n):
    return [(c0, min(n, c0 + BLK)) for c0 in range(0, n, BLK)]


def _lower(M, c0, c1, off):
    """Columns c0..c1-1 of M with only rows i >= column + off kept."""
    import torch
    return torch.tril(M[:, c0:c1], -(c0 + off))


@pytest.mark.parametrize("n,nb", [(50000, None), (98304, None), (40000, "16")])
def test_wide_order_properties(skf, n, nb, monkeypatch):
    import torch
    monkeypatch.delenv("SKF_NB", raising=False)
    if nb:
        monkeypatch.setenv("SKF_NB", nb)
    width = skf.tune_get("ltlt_nb", n)
    print(f"wide case n={n} panel width {width}", flush=True)
    assert width in (16, 32, 64) and (nb is None or width == int(nb))
    # Gaussian entries drawn on the device (seeded): only the strict lower
    # triangle is read, so the skew matrix is S - S^T with S that triangle
    dA = skf.colmajor(n, n)
    dA.normal_(generator=torch.Generator(device=dA.device).manual_seed(9000 + n))
    A0 = dA.clone()
    ipiv, T, info = skf.ltlt(dA)
    torch.cuda.synchronize()
    assert info == 0
    ip = ipiv.cpu().numpy()
    assert ip[0] == 0 and np.all(ip >= np.arange(n)) and np.all(ip < n)
    # the multipliers: column c of L (c >= 1) sits below the subdiagonal of column c - 1
    lmax = max(float(_lower(dA, c0, min(c1, n - 1), 2).abs().max()) for c0, c1 in _blocks(n - 1))
    assert lmax <= 1.0
    # reconstruction residual by probes: R v = P A P^T v - L T L^T v, with
    # A = S - S^T (S the strict lower triangle) and L = I + (the multipliers)
    a_fro = math.sqrt(2.0 * sum(float((_lower(A0, c0, c1, 1) ** 2).sum()) for c0, c1 in _blocks(n)))
    t = T[:n - 1]
    rng = np.random.default_rng(77)
    acc = 0.0
    nprobe = 4
    for _ in range(nprobe):
        v = rng.standard_normal(n)
        w = torch.from_numpy(_apply_P(v, ip, transpose=True)).to(dA.device)
        y = torch.zeros_like(w)
        for c0, c1 in _blocks(n):
            Sb = _lower(A0, c0, c1, 1)
            y += Sb @ w[c0:c1]
            y[c0:c1] -= Sb.T @ w
        y1 = _apply_P(y.cpu().numpy(), ip)
        vd = torch.from_numpy(v).to(dA.device)
        u = vd.clone()
        for c0, c1 in _blocks(n - 1):
            u[1 + c0:1 + c1] += _lower(dA, c0, c1, 2).T @ vd
        tu = torch.zeros_like(u)
        tu[1:] += t * u[:-1]
        tu[:-1] -= t * u[1:]
        z = tu.clone()
        for c0, c1 in _blocks(n - 1):
            z += _lower(dA, c0, c1, 2) @ tu[1 + c0:1 + c1]
        acc += float(np.sum((y1 - z.cpu().numpy()) ** 2))
    rel = np.sqrt(acc / nprobe) / (n * a_fro)
    print(f"n={n}: reconstruction residual {rel:.3e}", flush=True)
    assert rel <= RECON_TOL, rel
    # log|Pf| and sign from the factors against the Pfaffian-only reduction of
    # the same matrix (run last, on A0 itself: at n = 98304 three n x n copies
    # besides its workspace would not fit in HBM)
    la, sg = skf.logpf_from_factors(n, ipiv, T)
    la, sg = float(la.item()), int(sg.item())
    del dA
    torch.cuda.empty_cache()
    la2, sg2, info2 = skf.logpf(A0)
    la2, sg2 = float(la2.item()), int(sg2.item())
    print(f"n={n}: log|Pf| {la!r} vs Pfaffian-only {la2!r}", flush=True)
    assert info2 == 0 and sg == sg2
    assert abs(la - la2) <= LOGPF_TOL * max(1.0, abs(la))
