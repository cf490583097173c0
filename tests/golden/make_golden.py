"""Write the oracle's reference results for the large seeded workloads.

Calls only the generator and ``oracle/`` (never the GPU path).  Output per
(n, seed): ``ltlt_n{n}_s{seed}.npz`` with ipiv (int32), T (float64), logabs,
sign, info, the minimum relative pivot gap and the oracle's wall time.

    python tests/golden/make_golden.py 16384 2 [threads]
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


def main():
    n = int(sys.argv[1])
    seed = int(sys.argv[2])
    threads = int(sys.argv[3]) if len(sys.argv) > 3 else (os.cpu_count() or 1)
    A = inputs.skew_gaussian(n, seed, inputs.STREAM_A)
    t0 = time.time()
    f = oracle.ltlt(A, nthreads=threads, want_gap=True, inplace=True)
    dt = time.time() - t0
    la, sg = oracle.logpf_from_factors(n, f.ipiv, f.T)
    gap = f.gap if f.gap is not None and f.gap.size else np.ones(1)
    out = os.path.join(HERE, f"ltlt_n{n}_s{seed}.npz")
    np.savez(out, ipiv=f.ipiv.astype(np.int32), T=f.T.astype(np.float64), logabs=np.float64(la),
             sign=np.int32(sg), info=np.int32(f.info), min_gap=np.float64(gap.min()),
             argmin_gap=np.int64(int(np.argmin(gap))), oracle_seconds=np.float64(dt),
             oracle_threads=np.int32(threads))
    print(f"n={n} seed={seed} info={f.info} logabs={la!r} sign={sg} min_gap={gap.min():.3e} "
          f"time={dt:.1f}s threads={threads} -> {out}")


if __name__ == "__main__":
    main()
