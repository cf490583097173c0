"""Write the oracle's reference results for the large seeded workloads.

Calls only the generator and ``oracle/`` (never the GPU path).  Output per
(mode, n, seed):

* ``ltlt_n{n}_s{seed}.npz`` (full factorization): ipiv (int32), T (float64),
  T_mag (the magnitude sum of each T[k], for the per-entry tolerance), logabs,
  sign, info, the minimum relative pivot gap, the oracle's wall time and thread
  count, and a seeded sample of L: four whole columns (``Lcols`` indices,
  ``Lcol_vals`` / ``Lcol_mag`` of shape (4, n), rows above the diagonal zero)
  and 16384 single entries (``Li``, ``Lj``, ``Lvals``, ``Lmag``), where the
  magnitude sum is that of the multiplier's numerator;
* ``pfonly_n{n}_s{seed}.npz`` (Pfaffian-only reduction): ipiv, T, T_mag,
  logabs, sign, info, oracle wall time and threads;
* ``pfonly_c128_n{n}_s{seed}.npz`` (complex Pfaffian-only reduction of the
  complex skew Gaussian matrix of the same seed): ipiv, T (complex128), T_mag,
  logabs, phase, info, oracle wall time.

    python tests/golden/make_golden.py 16384 2 [threads] [ltlt|pfonly|c128]

When the file already exists, the new pivots and T must equal the stored ones
bit for bit (the oracle's arithmetic is deterministic), else nothing is written.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2408_05238_amd import inputs  # noqa: E402

N_LCOLS = 4
N_LENTRIES = 16384


def _check_same(out, ipiv, T):
    if not os.path.exists(out):
        return
    old = np.load(out)
    if not (np.array_equal(old["ipiv"], ipiv) and np.array_equal(old["T"], T)):
        raise SystemExit(f"{out}: new oracle results differ from the stored ones; not overwritten")
    print(f"{out}: pivots and T equal to the stored results bit for bit")


def _l_sample(n, seed, LT, M):
    rng = np.random.default_rng(1000 + seed)
    cols = np.sort(rng.choice(np.arange(1, n - 1), size=N_LCOLS, replace=False)).astype(np.int64)
    cv = np.zeros((N_LCOLS, n))
    cm = np.zeros((N_LCOLS, n))
    for t, j in enumerate(cols):  # L[i, j] (i > j) is stored at LT[i, j-1]
        cv[t, j + 1:] = LT[j + 1:, j - 1]
        cm[t, j + 1:] = M[j + 1:, j - 1]
    j = rng.integers(1, n - 1, size=N_LENTRIES)
    i = j + 1 + (rng.random(N_LENTRIES) * (n - 1 - j)).astype(np.int64)
    i = np.minimum(i, n - 1)
    return dict(Lcols=cols, Lcol_vals=cv, Lcol_mag=cm, Li=i.astype(np.int32), Lj=j.astype(np.int32),
                Lvals=LT[i, j - 1].copy(), Lmag=M[i, j - 1].copy())


def main():
    n = int(sys.argv[1])
    seed = int(sys.argv[2])
    threads = int(sys.argv[3]) if len(sys.argv) > 3 else (os.cpu_count() or 1)
    mode = sys.argv[4] if len(sys.argv) > 4 else "ltlt"
    if mode == "c128":
        A = inputs.skew_gaussian_c128(n, seed)
        t0 = time.time()
        ipiv, T, info, Tm = oracle.pfonly_c128(A, want_mag=True)
        dt = time.time() - t0
        la, ph = oracle.logpf_c128_from_factors(n, ipiv, T)
        out = os.path.join(HERE, f"pfonly_c128_n{n}_s{seed}.npz")
        if os.path.exists(out):
            old = np.load(out)
            if not (np.array_equal(old["ipiv"], ipiv) and np.array_equal(old["T"], T)):
                raise SystemExit(f"{out}: new oracle results differ from the stored ones; not overwritten")
        np.savez(out, ipiv=ipiv.astype(np.int32), T=T.astype(np.complex128), T_mag=Tm, logabs=np.float64(la),
                 phase=np.complex128(ph), info=np.int32(info), oracle_seconds=np.float64(dt))
        print(f"c128 n={n} seed={seed} info={info} logabs={la!r} phase={ph!r} time={dt:.1f}s -> {out}")
        return
    A = inputs.skew_gaussian(n, seed, inputs.STREAM_A)
    t0 = time.time()
    if mode == "pfonly":
        ipiv, T, info, Tm = oracle.pfonly(A, nthreads=threads, want_mag=True)
        dt = time.time() - t0
        del A
        la, sg = oracle.logpf_from_factors(n, ipiv, T)
        out = os.path.join(HERE, f"pfonly_n{n}_s{seed}.npz")
        _check_same(out, ipiv.astype(np.int32), T.astype(np.float64))
        np.savez(out, ipiv=ipiv.astype(np.int32), T=T.astype(np.float64), T_mag=Tm, logabs=np.float64(la),
                 sign=np.int32(sg), info=np.int32(info), oracle_seconds=np.float64(dt),
                 oracle_threads=np.int32(threads))
        print(f"pfonly n={n} seed={seed} info={info} logabs={la!r} sign={sg} time={dt:.1f}s "
              f"threads={threads} -> {out}")
        return
    f = oracle.ltlt(A, nthreads=threads, want_gap=True, inplace=True, want_mag=True)
    dt = time.time() - t0
    la, sg = oracle.logpf_from_factors(n, f.ipiv, f.T)
    gap = f.gap if f.gap is not None and f.gap.size else np.ones(1)
    out = os.path.join(HERE, f"ltlt_n{n}_s{seed}.npz")
    _check_same(out, f.ipiv.astype(np.int32), f.T.astype(np.float64))
    extra = _l_sample(n, seed, f.LT, f.M)
    np.savez(out, ipiv=f.ipiv.astype(np.int32), T=f.T.astype(np.float64), T_mag=f.T_mag(),
             logabs=np.float64(la), sign=np.int32(sg), info=np.int32(f.info), min_gap=np.float64(gap.min()),
             argmin_gap=np.int64(int(np.argmin(gap))), oracle_seconds=np.float64(dt),
             oracle_threads=np.int32(threads), **extra)
    print(f"n={n} seed={seed} info={f.info} logabs={la!r} sign={sg} min_gap={gap.min():.3e} "
          f"time={dt:.1f}s threads={threads} -> {out}")


if __name__ == "__main__":
    main()
