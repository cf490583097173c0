"""Seeded synthetic inputs (skew Gaussian matrices, right-hand sides, size mixes).

Thin ctypes layer over ``skgen.c``; see that file for the exact definition of
every draw.  Nothing here performs any step of the factorization: this module is
the only code shared between the GPU path's callers and the CPU oracle's tests.

Stream ids (the second key argument) used by the workloads:
    STREAM_A      = 0      single dense skew matrix
    STREAM_B      = 1      right-hand sides of a solve
    STREAM_SIZES  = 2      sizes of a batch
    STREAM_SERVE  = 3      serving request mix
    STREAM_IMAG   = 4      imaginary part of a complex skew matrix
    STREAM_BATCH0 = 1000   matrix b of a batch uses stream 1000 + b
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

STREAM_A = 0
STREAM_B = 1
STREAM_SIZES = 2
STREAM_SERVE = 3
STREAM_IMAG = 4
STREAM_BATCH0 = 1000

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libskgen.so")
_SRC_PATH = os.path.join(_HERE, "skgen.c")
_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile ``libskgen.so`` with gcc (strict IEEE: no contraction, no fast-math)."""
    import subprocess

    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
             "-std=c11", "-o", tmp, _SRC_PATH, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            i64, u64, dp = ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)
            lib.skgen_mix64.restype = u64
            lib.skgen_mix64.argtypes = [u64]
            lib.skgen_key.restype = u64
            lib.skgen_key.argtypes = [u64, u64]
            lib.skgen_gauss.restype = ctypes.c_double
            lib.skgen_gauss.argtypes = [u64, u64]
            lib.skgen_uniform.restype = ctypes.c_double
            lib.skgen_uniform.argtypes = [u64, u64]
            lib.skgen_log.restype = ctypes.c_double
            lib.skgen_log.argtypes = [ctypes.c_double]
            lib.skgen_skew_gaussian.argtypes = [i64, dp, i64, u64, u64]
            lib.skgen_skew_gaussian_cols.argtypes = [i64, dp, i64, u64, u64, i64, i64]
            lib.skgen_gaussian.argtypes = [i64, i64, dp, i64, u64, u64]
            lib.skgen_even_sizes.argtypes = [i64, i64, i64, ctypes.POINTER(ctypes.c_int64), u64, u64]
            _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def key(seed: int, stream: int) -> int:
    return int(_load().skgen_key(seed, stream))


def gauss(seed: int, stream: int, ctr: int) -> float:
    return float(_load().skgen_gauss(key(seed, stream), ctr))


def uniform(seed: int, stream: int, ctr: int) -> float:
    return float(_load().skgen_uniform(key(seed, stream), ctr))


def log(x: float) -> float:
    """The generator's own natural logarithm (exposed for its tests)."""
    return float(_load().skgen_log(x))


def skew_gaussian(n: int, seed: int, stream: int = STREAM_A, lda: int | None = None,
                  threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Column-major n x n skew matrix: A[i,j] ~ N(0,1) for i<j, A[j,i] = -A[i,j], A[i,i] = 0.

    Returns a Fortran-ordered float64 array of shape (lda, n) sliced to (n, n).
    """
    lib = _load()
    lda = n if lda is None else lda
    if out is None:
        buf = np.empty((lda, max(n, 1)), dtype=np.float64, order="F")
    else:
        buf = out
        assert buf.flags.f_contiguous and buf.shape[0] == lda and buf.dtype == np.float64
    if n == 0:
        return buf[:0, :0]
    nthr = threads if threads is not None else min(8, os.cpu_count() or 1)
    nthr = max(1, min(nthr, n))
    if nthr == 1 or n < 256:
        lib.skgen_skew_gaussian(n, _dptr(buf), lda, seed, stream)
    else:
        # column ranges balanced by work (column j costs n draws either way)
        bounds = np.linspace(0, n, nthr + 1).astype(np.int64)
        ths = [threading.Thread(target=lib.skgen_skew_gaussian_cols,
                                args=(n, _dptr(buf), lda, seed, stream, int(bounds[t]), int(bounds[t + 1])))
               for t in range(nthr)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
    return buf[:n, :n]


def skew_gaussian_c128(n: int, seed: int, threads: int = 8) -> np.ndarray:
    """Complex skew matrix: real part from STREAM_A, imaginary part from STREAM_IMAG."""
    re = skew_gaussian(n, seed, STREAM_A, threads=threads)
    im = skew_gaussian(n, seed, STREAM_IMAG, threads=threads)
    return re + 1j * im


def gaussian(rows: int, cols: int, seed: int, stream: int = STREAM_B) -> np.ndarray:
    """Column-major rows x cols block of N(0,1) draws (counter i + j*rows)."""
    buf = np.empty((max(rows, 1), max(cols, 1)), dtype=np.float64, order="F")
    if rows and cols:
        _load().skgen_gaussian(rows, cols, _dptr(buf), rows, seed, stream)
    return buf[:rows, :cols]


def even_sizes(count: int, nmin: int, nmax: int, seed: int, stream: int = STREAM_SIZES) -> np.ndarray:
    """Even sizes uniform on {nmin, nmin+2, ..., nmax}."""
    assert nmin % 2 == 0 and nmax % 2 == 0 and nmin <= nmax
    out = np.empty(max(count, 1), dtype=np.int64)
    _load().skgen_even_sizes(count, nmin, nmax, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             seed, stream)
    return out[:count]


def batch_matrix(n: int, seed: int, b: int) -> np.ndarray:
    """Matrix b of a batch (its own stream STREAM_BATCH0 + b)."""
    return skew_gaussian(n, seed, STREAM_BATCH0 + b, threads=1)
