"""Parity at the full benchmark sizes: n = 16384 FP64 with seeds 2, 3 and 4, in
the launch configuration bench.py times (skf.ltlt, default block size), seed 2
again with the narrow panel (nb = 64) and the widest one (nb = 256, one panel
workgroup per CU), and the n = 32768 matrix of the mixed
precision workload (seed 5) at both widths: nb = 128 (512 panel workgroups, two
per CU: the tuned choice) and nb = 64 (512 workgroups of the narrow panel).

The reference is the oracle's own result for the same seeded input, stored in
tests/golden/ltlt_n16384_s{seed}.npz by tests/golden/make_golden.py (which calls
only the generator and the oracle): the interchanges are compared bit for bit,
T and a stored sample of L entry by entry within the summation-error bound of
each entry's magnitude sum, log|Pf| within 1e-12.  The reconstruction residual
||P A P^T - L T L^T||_F / (n ||A||_F) is estimated on the device in FP64 with
Gaussian probe vectors (E ||R v||^2 = ||R||_F^2 for v with independent N(0,1)
entries), the interchanges applied on the host.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
N = 16384
# T and L: same interchanges, different rounding (blocked paired updates with
# FMA and matrix-core products vs the unblocked update without contraction).
# Each entry is compared within the summation-error bound of its own magnitude
# sum, stored by make_golden.py (oracle.t_tolerance / oracle.l_tolerance).
LOGPF_TOL = 1e-12    # |d log|Pf|| / max(1, |log|Pf||)
RECON_TOL = 1e-13    # ||PAP^T - LTL^T||_F / (n ||A||_F)


@pytest.fixture(scope="module")
def skf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_05238_amd import skf as s
    s.lib()
    return s


def _apply_P(x, ipiv, transpose=False):
    """P x (interchanges j <-> ipiv[j] for j = 1..n-1 in order) or P^T x (reverse order)."""
    x = x.copy()
    js = range(len(ipiv) - 1, 0, -1) if transpose else range(1, len(ipiv))
    for j in js:
        p = int(ipiv[j])
        if p != j:
            x[[j, p]] = x[[p, j]]
    return x


CASES = [(N, 2, None), (N, 3, None), (N, 4, None), (N, 2, "64"), (N, 2, "256"), (32768, 5, None), (32768, 5, "64")]


@pytest.mark.parametrize("n,seed,nb", CASES, ids=[f"n{c[0]}-s{c[1]}-nb{c[2] or 'auto'}" for c in CASES])
def test_ltlt_fullsize_against_stored_oracle(skf, n, seed, nb, monkeypatch):
    """n = 16384 in the launch configuration bench.py times (nb = 128, 256 panel
    workgroups), the same matrix with the narrow panel (nb = 64: 256 workgroups),
    and n = 32768 (512 workgroups) at nb = 128 and nb = 64."""
    import torch
    import oracle
    from paper_2408_05238_amd import inputs
    if nb:
        monkeypatch.setenv("SKF_NB", nb)
    path = os.path.join(HERE, "golden", f"ltlt_n{n}_s{seed}.npz")
    assert os.path.exists(path), path
    g = np.load(path)
    print(f"case n={n} seed={seed} nb={nb or 'auto'}", flush=True)
    A = inputs.skew_gaussian(n, seed, inputs.STREAM_A)
    dA = skf.to_device_colmajor(A)
    del A
    A0 = dA.clone()
    ipiv, T, info = skf.ltlt(dA)
    torch.cuda.synchronize()
    assert info == int(g["info"]) == 0
    ip = ipiv.cpu().numpy()
    assert np.array_equal(ip, g["ipiv"]), int(np.argmax(ip != g["ipiv"]))
    Th = T.cpu().numpy()[:n - 1]
    d = np.abs(Th - g["T"])
    tol = oracle.t_tolerance(g["T_mag"])
    k = int(np.argmax(d / tol))
    print(f"seed {seed}: max |dT| / bound = {d[k] / tol[k]:.3e} at k = {k} (T = {g['T'][k]!r}); "
          f"max |dT| / max |T| = {d.max() / np.abs(g['T']).max():.3e}; min pivot gap {float(g['min_gap']):.3e}")
    assert np.all(d <= tol), int(np.argmax(d - tol))
    la, sg = skf.logpf_from_factors(n, ipiv, T)
    print(f"seed {seed}: log|Pf| {la!r} vs {float(g['logabs'])!r}")
    assert sg == int(g["sign"])
    assert abs(la - float(g["logabs"])) <= LOGPF_TOL * max(1.0, abs(float(g["logabs"])))

    # L: the stored sample of whole columns and single entries, entry by entry
    tm = g["T_mag"]
    for t, j in enumerate(g["Lcols"]):
        j = int(j)
        got = dA[j + 1:, j - 1].cpu().numpy()
        ref = g["Lcol_vals"][t, j + 1:]
        tl = oracle.l_tolerance(ref, g["Lcol_mag"][t, j + 1:], g["T"][j - 1], tm[j - 1], j)
        assert np.all(np.abs(got - ref) <= tl), (j, float(np.abs(got - ref).max()))
    li = torch.from_numpy(g["Li"].astype(np.int64)).to(dA.device)
    lj = torch.from_numpy(g["Lj"].astype(np.int64) - 1).to(dA.device)
    got = dA[li, lj].cpu().numpy()
    jj = g["Lj"].astype(np.int64)
    tl = oracle.l_tolerance(g["Lvals"], g["Lmag"], g["T"][jj - 1], tm[jj - 1], jj)
    dl = np.abs(got - g["Lvals"])
    print(f"seed {seed}: L sample max |dL| / bound = {(dl / tl).max():.3e}")
    assert np.all(dl <= tl)

    # reconstruction residual by probes: R v = P A P^T v - L T L^T v
    N_ = n
    S = torch.tril(A0, -1)                 # A = S - S^T
    del A0
    a_fro = float(torch.sqrt(2.0 * (S * S).sum()))
    Ls = torch.tril(dA, -2)[:, :-1]        # column j-1 holds L[:, j] below its diagonal, j >= 1
    t = T[:N_ - 1]
    rng = np.random.default_rng(1000 + seed)
    nprobe = 8
    acc = 0.0
    for _ in range(nprobe):
        v = rng.standard_normal(N_)
        w = torch.from_numpy(_apply_P(v, ip, transpose=True)).to(dA.device)
        y = (S @ w - S.T @ w).cpu().numpy()
        y1 = _apply_P(y, ip)
        vd = torch.from_numpy(v).to(dA.device)
        u = vd.clone()
        u[1:] += Ls.T @ vd                 # L^T v
        tu = torch.zeros_like(u)
        tu[1:] += t * u[:-1]               # T u: sub-diagonal t, super-diagonal -t
        tu[:-1] -= t * u[1:]
        z = tu + Ls @ tu[1:]               # L (T L^T v)
        acc += float(np.sum((y1 - z.cpu().numpy()) ** 2))
    rel = np.sqrt(acc / nprobe) / (N_ * a_fro)
    assert rel <= RECON_TOL, rel
